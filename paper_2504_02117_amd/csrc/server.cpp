// The serving loop: a worker thread with its own stream admits requests in arrival order as HBM
// budget and slots allow, keeps every admitted solve's state resident on the device, and advances
// all of them round by round.  A round enqueues the outer-loop work of the jobs that need it (the
// FP64 all-at-once residual, the scaled FP32 restart, the correction Y -= V), then ONE grouped
// launch per block-CG kernel and block-width class for every job inside its inner solve, then one
// read-back of all jobs' norms.  Requests that arrive while others run join at the next round.
//
// A mode-0 request solves the all-at-once system of one window of k columns (Sec. 2.1, eq.
// general-system-time-steps) by the Newton/splitting iteration of eq. matrix-fixed-point-equation,
// until every column meets the tolerance; the inner solves are FP32 block CG with Jacobi, the
// residual and the update are FP64.  A mode-1 request runs the pipelined Algorithm 1 (its front
// column accepted as soon as it converges) with multigrid-preconditioned block CG on a lane of its
// own: up to kLanes threads, each with a context and stream, take mode-1 requests from the same
// arrival-order queue under the same HBM budget.
#include "server.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>

#include "advance.hpp"
#include "serve.hpp"
#include "timecoupling.hpp"
#include "vecops.hpp"
#include "wide.hpp"

namespace bkts {
bkts_op fv_assemble(bkts_ctx ctx, const bkts_grid* grid, const bkts_fv_coeffs* c, int format);
void set_last_error(const std::string& m);
}  // namespace bkts

using namespace bkts;

namespace {

constexpr int kStatusStride = 4 * BKTS_MAX_K;  // doubles per slot: nrm64 | nrm | nrm0 | ndefl

// Padded width of a job: row-tile kernels up to 4 columns, the FP32 matrix-core kernels beyond.
int kp_of(int k) { return k <= 1 ? 1 : k <= 2 ? 2 : k <= 4 ? 4 : wide_kp(k); }

int64_t grid_cells(const bkts_grid& g) {
  int64_t n = 1;
  for (int d = 0; d < g.dim; ++d) n *= g.n[d];
  return n;
}

}  // namespace

size_t bkts_server_s::footprint(const bkts_request& r) {
  const int64_t N = grid_cells(r.grid);
  const int64_t nnz = (2 * r.grid.dim + 1) * N;
  const int k = r.k, kp = kp_of(k);
  int64_t tps;
  const int ns = gjob_slots(N, kp, &tps);
  size_t b = 0;
  b += 4 * (N + 1) + nnz * (4 + 8 + 4) + 16 * N;        // CSR, FP32 values, diagonal, b
  b += (size_t)(nnz * 1.1) * (4 + 8 + 4) + 16 * (N / 64 + 1);  // SELL copy
  b += 16 * (N + 1);                                    // assembly scratch
  b += (size_t)N * k * (8 + 8 + 4 * 4);                 // Y, R (FP64), X, P, Q, R (FP32)
  b += (size_t)N * 8 * (1 + 3);                         // dinv, B0 (up to 3 columns)
  b += (size_t)8 * ns * (2 * kp * kp + kp);             // partials
  b += 8 * (8 * BKTS_MAX_K * BKTS_MAX_K);               // k x k buffers
  return b;
}

// Mode 1: the operator (CSR with its FP32 values, the stencil form in FP64 and FP32), the
// multigrid hierarchy (five coefficient arrays and an inverse diagonal in both precisions, about
// 8/7 of the fine level in total), the pipeline window (Y, R, V and the stage history), the FP32
// block-CG blocks (R, P, Q, Z, the scaled residual and correction), the multigrid level buffers,
// the accepted steps (k x N) and small buffers.
size_t bkts_server_s::footprint_pipelined(const bkts_request& r) {
  const int64_t N = grid_cells(r.grid);
  const int64_t nnz = (2 * r.grid.dim + 1) * N;
  const int w = r.window > 0 ? r.window : std::min(r.k, 4);
  size_t b = 0;
  b += 4 * (N + 1) + nnz * (4 + 8 + 4) + 16 * N + 16 * (N + 1);  // CSR, diagonal, b, assembly scratch
  b += (size_t)(1 + r.grid.dim) * N * (8 + 4);                    // stencil form
  b += (size_t)(N * 8 / 7 + 64) * 6 * (8 + 4);                     // multigrid hierarchy
  b += (size_t)N * w * 8 * 3 + (size_t)N * 8 * 6;                  // window, residual, correction, history
  b += (size_t)N * w * 4 * 6 + (size_t)(N * 8 / 7 + 64) * w * 4 * 2;  // FP32 block CG, level buffers
  b += (size_t)N * r.k * 8 + (size_t)N * 8;                        // accepted steps, y
  b += (size_t)1 << 20;                                            // k x k buffers and partials
  return b;
}

bkts_server_s::bkts_server_s(int device, size_t budget_, int max_slots_)
    : budget(budget_), max_slots(max_slots_), t0(std::chrono::steady_clock::now()) {
  BKTS_HIP(hipSetDevice(device));
  hipStream_t s = nullptr;
  BKTS_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
  ctx = new bkts_ctx_s();
  ctx->device = device;
  ctx->stream = s;
  int ncu = 0;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && ncu > 0)
    ctx->num_cu = ncu;
  jobs.resize(max_slots);
  status_dev.alloc(sizeof(double) * kStatusStride * max_slots);
  BKTS_HIP(hipHostMalloc(reinterpret_cast<void**>(&status_host), sizeof(double) * kStatusStride * max_slots,
                         hipHostMallocDefault));
  table_bytes = sizeof(GJob) * max_slots + sizeof(int) * 16 * (max_slots + 1) * 4;
  table_dev.alloc(table_bytes);
  BKTS_HIP(hipHostMalloc(&table_host, table_bytes, hipHostMallocDefault));
  nlanes = std::min(kLanes, max_slots);
  for (int l = 0; l < nlanes; ++l) {
    Lane& L = lanes[l];
    hipStream_t ls = nullptr;
    BKTS_HIP(hipStreamCreateWithFlags(&ls, hipStreamNonBlocking));  // default priority
    L.ctx = new bkts_ctx_s();
    L.ctx->device = device;
    L.ctx->stream = ls;
    L.ctx->num_cu = ctx->num_cu;
  }
  worker = std::thread([this] { run(); });
  for (int l = 0; l < nlanes; ++l) lanes[l].th = std::thread([this, l] { lane_run(l); });
}

bkts_server_s::~bkts_server_s() {
  {
    std::lock_guard<std::mutex> g(mu);
    stop = true;
  }
  cv.notify_all();
  if (worker.joinable()) worker.join();
  for (Lane& L : lanes)
    if (L.th.joinable()) L.th.join();
  for (Lane& L : lanes) {
    if (!L.ctx) continue;
    (void)hipStreamSynchronize(L.ctx->stream);
    L.ctx->ws.bufs.clear();
    if (L.ctx->h_pinned) (void)hipHostFree(L.ctx->h_pinned);
    (void)hipStreamDestroy(L.ctx->stream);
    delete L.ctx;
    L.ctx = nullptr;
  }
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  for (auto& j : jobs) j.reset();
  status_dev.release();
  table_dev.release();
  if (status_host) (void)hipHostFree(status_host);
  if (table_host) (void)hipHostFree(table_host);
  ctx->ws.bufs.clear();
  if (ctx->h_pinned) (void)hipHostFree(ctx->h_pinned);
  (void)hipStreamDestroy(ctx->stream);
  delete ctx;
}

double bkts_server_s::now() const {
  return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

uint64_t bkts_server_s::submit(const bkts_request& r) {
  BKTS_REQUIRE(r.grid.dim >= 1 && r.grid.dim <= 3, "request grid dim must be 1..3");
  for (int d = 0; d < r.grid.dim; ++d) BKTS_REQUIRE(r.grid.n[d] >= 1, "request grid n[%d] < 1", d);
  BKTS_REQUIRE(r.k >= 1 && r.k <= BKTS_MAX_K, "request k must be in 1..%d", BKTS_MAX_K);
  BKTS_REQUIRE(r.tau > 0.0, "request tau must be > 0");
  BKTS_REQUIRE(r.rtol > 0.0 && r.rtol < 1.0, "request rtol must be in (0, 1)");
  BKTS_REQUIRE(r.inner_rtol > 0.0 && r.inner_rtol < 1.0, "request inner_rtol must be in (0, 1)");
  BKTS_REQUIRE(r.y0 && r.y_out, "request y0 and y_out must not be NULL");
  BKTS_REQUIRE(r.method == BKTS_IE || r.method == BKTS_THETA || r.method == BKTS_SDIRK2,
               "request method must be BKTS_IE, BKTS_THETA or BKTS_SDIRK2");
  BKTS_REQUIRE(r.mode == 0 || r.mode == 1, "request mode must be 0 (grouped) or 1 (pipelined)");
  BKTS_REQUIRE(r.mode == 0 || r.method == BKTS_IE, "pipelined (mode 1) requests take implicit Euler");
  BKTS_REQUIRE(r.window >= 0 && r.window <= r.k, "request window must be in 0..k");
  BKTS_REQUIRE(grid_cells(r.grid) < (int64_t)1 << 30, "request grid too large");
  const size_t fp = r.mode == 1 ? footprint_pipelined(r) : footprint(r);
  if (fp > budget)
    throw Error{BKTS_ENOMEM, fmt("request needs %.1f MB, more than the server budget of %.1f MB", fp / 1e6,
                                 budget / 1e6)};
  std::lock_guard<std::mutex> g(mu);
  BKTS_REQUIRE(!stop, "server is shutting down");
  Pending p;
  p.req = r;
  p.ticket = ++next_ticket;
  p.t_submit = now();
  p.footprint = fp;
  queue.push_back(p);
  cv.notify_all();
  return p.ticket;
}

int bkts_server_s::poll(bkts_result* out, int max) {
  std::lock_guard<std::mutex> g(mu);
  int n = 0;
  while (n < max && !done.empty()) {
    out[n++] = done.front();
    done.pop_front();
  }
  return n;
}

int bkts_server_s::wait(int n, double timeout_s) {
  std::unique_lock<std::mutex> g(mu);
  const auto until = std::chrono::steady_clock::now() + std::chrono::duration<double>(timeout_s);
  cv_done.wait_until(g, until, [&] { return (int)done.size() >= n || fatal; });
  return (int)done.size();
}

bkts_server_stats bkts_server_s::stats() {
  std::lock_guard<std::mutex> g(mu);
  bkts_server_stats s{};
  s.queued = (int)queue.size();
  s.active = n_active;
  s.done_unpolled = (int)done.size();
  s.rounds = rounds;
  s.grouped_launches = grouped_launches;
  s.bytes_in_use = in_use;
  s.bytes_peak = peak;
  s.max_active = max_active;
  return s;
}

// ------------------------------------------------------------------ worker

void bkts_server_s::run() {
  (void)hipSetDevice(ctx->device);
  try {
    for (;;) {
      std::vector<std::pair<int, Pending>> admit;
      {
        std::unique_lock<std::mutex> g(mu);
        if (n_active == 0 && queue.empty()) {
          if (stop) break;
          cv.wait_for(g, std::chrono::milliseconds(2));
          continue;
        }
        // strict arrival order: the head waits until it fits
        while (!queue.empty() && !stop) {
          const Pending& h = queue.front();
          if (in_use + h.footprint > budget) break;
          if (h.req.mode == 1) {  // a pipelined request goes to a free lane
            int lane = -1;
            for (int l = 0; l < nlanes; ++l)
              if (!lanes[l].busy) {
                lane = l;
                break;
              }
            if (lane < 0) break;
            in_use += h.footprint;
            peak = std::max(peak, in_use);
            ++n_active;
            max_active = std::max(max_active, n_active);
            lanes[lane].busy = true;
            lanes[lane].p = h;
            queue.pop_front();
            cv.notify_all();
            continue;
          }
          int slot = -1;
          for (int s = 0; s < max_slots; ++s)
            if (!jobs[s] && std::find_if(admit.begin(), admit.end(), [&](auto& a) { return a.first == s; }) ==
                                admit.end()) {
              slot = s;
              break;
            }
          if (slot < 0) break;
          in_use += h.footprint;
          peak = std::max(peak, in_use);
          admit.emplace_back(slot, h);
          queue.pop_front();
        }
        if (stop) queue.clear();
      }
      for (auto& a : admit) setup(a.first, a.second);
      if (n_active_now() > 0) {
        round();
      } else {  // only lanes are busy, or the queue head waits for memory: sleep until something changes
        std::unique_lock<std::mutex> g(mu);
        if (!stop) cv.wait_for(g, std::chrono::milliseconds(2));
      }
    }
  } catch (const Error& e) {
    std::lock_guard<std::mutex> g(mu);
    fatal = true;
    fatal_msg = e.msg;
    cv_done.notify_all();
  } catch (const std::exception& e) {
    std::lock_guard<std::mutex> g(mu);
    fatal = true;
    fatal_msg = e.what();
    cv_done.notify_all();
  }
}

void bkts_server_s::lane_run(int l) {
  Lane& L = lanes[l];
  (void)hipSetDevice(L.ctx->device);
  for (;;) {
    Pending p;
    {
      std::unique_lock<std::mutex> g(mu);
      cv.wait(g, [&] { return (L.busy && L.p.ticket != 0) || (stop && !L.busy) || fatal; });
      if (!L.busy || fatal) {
        if (fatal && L.busy) L.busy = false;
        if (stop || fatal) return;
        continue;
      }
      p = L.p;
    }
    bkts_result res{};
    bool device_error = false;
    std::string msg;
    try {
      res = lane_solve(L, p);
    } catch (const Error& e) {
      device_error = e.status == BKTS_EDEVICE;
      msg = e.msg;
      res.ticket = p.ticket;
      res.tag = p.req.tag;
      res.status = e.status;
      res.t_submit = p.t_submit;
      res.t_done = now();
      res.footprint_bytes = p.footprint;
    }
    std::lock_guard<std::mutex> g(mu);
    in_use -= p.footprint;
    --n_active;
    L.busy = false;
    L.p = Pending{};
    if (device_error) {
      fatal = true;
      fatal_msg = msg;
    } else {
      done.push_back(res);
    }
    cv_done.notify_all();
    cv.notify_all();
  }
}

// Mode 1: the pipelined Algorithm 1 (implicit Euler, window of `window` columns) with FP32 block CG
// preconditioned by the multigrid V-cycle on the stencil form, then the k accepted steps written as
// the columns of y_out.  The lane's workspace is released afterwards, with the request's footprint.
bkts_result bkts_server_s::lane_solve(Lane& L, const Pending& p) {
  bkts_ctx c = L.ctx;
  const bkts_request& r = p.req;
  bkts_result res{};
  res.ticket = p.ticket;
  res.tag = r.tag;
  res.t_submit = p.t_submit;
  res.t_admit = now();
  res.footprint_bytes = p.footprint;
  struct Cleanup {
    bkts_ctx c;
    ~Cleanup() {
      (void)hipStreamSynchronize(c->stream);
      c->ws.bufs.clear();
    }
  } cleanup{c};
  bkts_fv_coeffs co{};
  co.kappa = r.kappa;
  co.kappa_const = r.kappa_const;
  for (int f = 0; f < 6; ++f) {
    co.bc_type[f] = r.bc_type[f];
    co.bc_value[f] = r.bc_value[f];
  }
  try {
    std::unique_ptr<bkts_op_s, OpDel> op(fv_assemble(c, &r.grid, &co, BKTS_FMT_STENCIL));
    bkts_tc_desc d{};
    d.method = BKTS_IE;
    d.k = r.window > 0 ? r.window : std::min(r.k, 4);
    d.tau = r.tau;
    std::unique_ptr<bkts_tc_s, TcDel> tc(tc_create(c, &d));
    const int64_t N = op->N;
    double* y = c->ws.get<double>("lane_y", N);
    double* hist = c->ws.get<double>("lane_hist", (size_t)N * r.k);
    BKTS_HIP(hipMemcpyAsync(y, r.y0, sizeof(double) * N, hipMemcpyDeviceToDevice, c->stream));
    bkts_solve_opts in{};
    in.krylov = BKTS_CG;
    in.precond = BKTS_PREC_MG;
    in.precision = BKTS_PRECISION_F32_REFINE;
    in.rtol = r.inner_rtol;
    in.inner_rtol = r.inner_rtol;
    in.maxit = r.max_inner > 0 ? r.max_inner : 100000;
    in.restart = 30;
    bkts_run_info ri{};
    const bkts_status st = advance(c, op.get(), tc.get(), y, r.k, in, r.rtol, r.max_outer > 0 ? r.max_outer : 200,
                                   hist, nullptr, nullptr, &ri);
    for (int j = 0; j < r.k && j < ri.accepted_steps; ++j) {  // step j + 1 into column j of y_out
      LinComb lc;
      lc.add(1.0, hist + (size_t)j * N, 1);
      lincomb(c, N, lc, r.y_out + j, r.k);
    }
    c->sync();
    res.status = st;
    res.outer_iterations = ri.outer_iterations;
    res.krylov_iterations = ri.krylov_iterations;
    res.rel_residual = ri.final_front_rel_residual;
  } catch (const Error& e) {
    if (e.status == BKTS_EDEVICE) throw;
    res.status = e.status;
  }
  res.t_done = now();
  return res;
}

int bkts_server_s::n_active_now() {
  int n = 0;
  for (auto& j : jobs) n += j ? 1 : 0;
  return n;
}

void bkts_server_s::setup(int slot, const Pending& p) {
  auto J = std::make_unique<Job>();
  J->p = p;
  J->t_admit = now();
  const bkts_request& r = p.req;
  try {
    bkts_fv_coeffs c{};
    c.kappa = r.kappa;
    c.kappa_const = r.kappa_const;
    for (int f = 0; f < 6; ++f) {
      c.bc_type[f] = r.bc_type[f];
      c.bc_value[f] = r.bc_value[f];
    }
    J->op.reset(fv_assemble(ctx, &r.grid, &c, BKTS_FMT_CSR));
    bkts_tc_desc d{};
    d.method = r.method;
    d.theta = r.theta;
    d.k = r.k;
    d.tau = r.tau;
    J->tc.reset(tc_create(ctx, &d));
    const int64_t N = J->op->N;
    const int k = r.k, kp = kp_of(k);
    const int mi = J->tc->m_impl;
    J->N = N;
    J->k = k;
    J->kp = kp;
    J->nb0 = std::min(mi, k);
    J->beta = J->tc->A2[0][0];
    int64_t tps;
    const int ns = gjob_slots(N, kp, &tps);
    const size_t nk = (size_t)N * k;
    J->Y.alloc(8 * nk);
    J->R64.alloc(8 * nk);
    J->f32.alloc(4 * nk * 4);
    J->dinv.alloc(8 * N);
    J->B0.alloc(8 * N * J->nb0);
    J->part.alloc(8 * (size_t)ns * (2 * kp * kp + kp));
    J->small.alloc(8 * (size_t)(6 * k * k + 2 * k + 2 * k * k + k));
    double* sm = J->small.as<double>();
    float* f = J->f32.as<float>();
    GJob& g = J->g;
    g.N = N;
    g.k = k;
    g.kp = kp;
    g.nslots = ns;
    g.tps = tps;
    g.a = 1.0 / r.tau;
    g.b = J->beta;
    g.rowptr = J->op->rowptr.as<int32_t>();
    g.col = J->op->col.as<int32_t>();
    g.val = J->op->val32.as<float>();
    g.dinv = J->dinv.as<double>();
    g.X = f;
    g.P = f + nk;
    g.Q = f + 2 * nk;
    g.R = f + 3 * nk;
    g.G = sm;
    g.gamma = sm + k * k;
    g.T = sm + 2 * k * k;
    g.alpha = sm + 3 * k * k;
    g.beta = sm + 4 * k * k;
    J->sc = sm + 5 * k * k;
    J->sp = J->sc + k;
    J->mats = J->sp + k;  // 2 k^2 + k
    double* st = status_dev.as<double>() + (size_t)slot * kStatusStride;
    J->nrm64 = st;
    g.nrm = st + k;
    J->nrm0 = st + 2 * k;
    g.ndefl = reinterpret_cast<int*>(st + 3 * k);
    g.pg = J->part.as<double>();
    g.pt = g.pg + (size_t)ns * kp * kp;
    g.pn = g.pt + (size_t)ns * kp * kp;
    jacobi_inverse(ctx, *J->op, g.a, g.b, J->dinv.as<double>());
    upload_window(ctx, *J->tc, 0, 0, J->mats, J->mats + k * k, J->mats + 2 * k * k);
    broadcast_cols(ctx, N, k, r.y0, J->Y.as<double>(), k);
    // B0 of the window starting at stage 0 (Sec. 2.2): y0/tau, minus the eliminated explicit stage
    double* fyn = nullptr;
    if (J->tc->explicit_first) {
      fyn = J->R64.as<double>();  // scratch until the first residual
      const double* bsrc = J->op->b_nonzero ? J->op->b.as<double>() : nullptr;
      spmm(ctx, *J->op, BKTS_F64, 1, -1.0, bsrc, 1, 0.0, r.y0, 1, 1.0, fyn, 1);
    }
    for (int q = 0; q < J->nb0; ++q) {
      LinComb lc;
      lc.add(1.0 / r.tau, r.y0, 1);
      if (fyn) lc.add(-J->tc->ae[q], fyn, 1);
      lincomb(ctx, N, lc, J->B0.as<double>() + q, J->nb0);
    }
    // scale of the equations: ||front column of B A2^T + B0||
    {
      double rs0 = 0.0;
      for (int j = 0; j < k; ++j) rs0 += J->tc->A2[0][j];
      LinComb lc;
      if (J->op->b_nonzero) lc.add(rs0, J->op->b.as<double>(), 1);
      lc.add(1.0, J->B0.as<double>(), J->nb0);
      double* tmp = J->R64.as<double>() + N;  // scratch
      if (k == 1) tmp = J->f32.as<double>();
      lincomb(ctx, N, lc, tmp, 1);
      colnorms2(ctx, BKTS_F64, N, 1, tmp, 1, J->nrm64);
      double h = 0.0;
      BKTS_HIP(hipMemcpyAsync(&h, J->nrm64, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
      ctx->sync();
      J->rhs0 = std::sqrt(h);
    }
    J->state = Job::RESID;
  } catch (const Error& e) {
    bkts_result res{};
    res.ticket = p.ticket;
    res.tag = p.req.tag;
    res.status = e.status;
    res.t_submit = p.t_submit;
    res.t_admit = J->t_admit;
    res.t_done = now();
    res.footprint_bytes = p.footprint;
    ctx->sync();
    J.reset();
    std::lock_guard<std::mutex> g(mu);
    in_use -= p.footprint;
    done.push_back(res);
    cv_done.notify_all();
    return;
  }
  jobs[slot] = std::move(J);
  std::lock_guard<std::mutex> g(mu);
  ++n_active;
  max_active = std::max(max_active, n_active);
}

void bkts_server_s::round() {
  const int n = max_slots;
  std::vector<int> resid, init, cg;
  int hi = 0;
  for (int s = 0; s < n; ++s) {
    Job* J = jobs[s].get();
    if (!J) continue;
    hi = s + 1;
    if (J->state == Job::RESID) resid.push_back(s);
    else if (J->state == Job::INIT) init.push_back(s);
    else if (J->state == Job::CG) cg.push_back(s);
  }
  // outer-loop work of single jobs
  for (int s : resid) {
    Job& J = *jobs[s];
    if (J.pending_apply)  // Y -= V, with V = -sp * X
      block_cast_scale(ctx, J.N, J.k, BKTS_F32, J.g.X, J.k, BKTS_F64, J.Y.as<double>(), J.k, J.sp, false, true);
    J.pending_apply = false;
    int cols[8];
    for (int i = 0; i < 8; ++i) cols[i] = i;
    residual(ctx, *J.op, J.k, J.Y.as<double>(), J.k, J.mats, J.mats + J.k * J.k, J.mats + 2 * J.k * J.k,
             J.B0.as<double>(), J.nb0, J.nb0, cols, J.R64.as<double>(), J.k, J.nrm64);
  }
  for (int s : init) {
    Job& J = *jobs[s];
    const int64_t N = J.N;
    const int k = J.k;
    scales_from_norms(ctx, k, J.nrm64, J.sc, J.sp);
    block_cast_scale(ctx, N, k, BKTS_F64, J.R64.as<double>(), k, BKTS_F32, J.g.R, k, J.sc, true, false);
    BKTS_HIP(hipMemsetAsync(J.g.X, 0, sizeof(float) * N * k, ctx->stream));
    cg_pupdate(ctx, BKTS_F32, N, k, J.g.P, J.g.R, nullptr, J.g.dinv);
    gram(ctx, BKTS_F32, N, k, J.g.R, k, J.g.P, k, J.g.gamma);
    colnorms2(ctx, BKTS_F32, N, k, J.g.R, k, J.nrm0);
    J.inner_it = 0;
    J.state = Job::CG;
    cg.push_back(s);
  }
  // one block-CG iteration of every job in an inner solve, grouped
  if (!cg.empty()) {
    std::sort(cg.begin(), cg.end());
    // host image of the table: jobs | per class (ids, first) | all (ids, first-blocks for G,
    // first-entries for G, first-entries for updates)
    GJob* hjobs = static_cast<GJob*>(table_host);
    for (int s : cg) hjobs[s] = jobs[s]->g;
    int* ib = reinterpret_cast<int*>(hjobs + max_slots);
    int* cur = ib;
    auto put = [&](const std::vector<int>& ids, auto count) {
      GList l{};
      int* pid = cur;
      for (size_t i = 0; i < ids.size(); ++i) pid[i] = ids[i];
      cur += ids.size();
      int* pf = cur;
      int acc = 0;
      for (size_t i = 0; i < ids.size(); ++i) {
        pf[i] = acc;
        acc += count(*jobs[ids[i]]);
      }
      pf[ids.size()] = acc;
      cur += ids.size() + 1;
      l.n = (int)ids.size();
      l.total = acc;
      l.ids = reinterpret_cast<const int*>(static_cast<char*>(table_dev.p) + (reinterpret_cast<char*>(pid) -
                                                                              static_cast<char*>(table_host)));
      l.first = reinterpret_cast<const int*>(static_cast<char*>(table_dev.p) + (reinterpret_cast<char*>(pf) -
                                                                                static_cast<char*>(table_host)));
      return l;
    };
    int classes[6] = {1, 2, 4, 8, 16, 32};
    GList cl[6];
    bool has[6] = {false, false, false, false, false, false};
    for (int c = 0; c < 6; ++c) {
      std::vector<int> ids;
      for (int s : cg)
        if (jobs[s]->kp == classes[c]) ids.push_back(s);
      if (ids.empty()) continue;
      has[c] = true;
      cl[c] = put(ids, [](const Job& J) { return J.g.nslots; });
    }
    GList lg = put(cg, [](const Job& J) { return J.k * J.k; });
    GList lu = put(cg, [](const Job& J) { return 2 * J.k * J.k + J.k; });
    GList ls = put(cg, [](const Job&) { return 1; });
    const size_t used = reinterpret_cast<char*>(cur) - static_cast<char*>(table_host);
    BKTS_REQUIRE(used <= table_bytes, "serving table overflow");
    BKTS_HIP(hipMemcpyAsync(table_dev.p, table_host, used, hipMemcpyHostToDevice, ctx->stream));
    const GJob* dj = table_dev.as<GJob>();
    const double eps = cg_pivot_floor(BKTS_F32);
    long nl = 0;
    // widths 16 and 32 run on the FP32 matrix cores, narrower ones on row tiles
    for (int c = 0; c < 6; ++c)
      if (has[c]) {
        if (classes[c] >= 16) gw_spmm_gram(ctx, classes[c] / 16, dj, cl[c]);
        else g_spmm_gram(ctx, classes[c], dj, cl[c]);
        ++nl;
      }
    g_finalize(ctx, 0, dj, lg);
    g_solve(ctx, 0, eps, dj, ls);
    for (int c = 0; c < 6; ++c)
      if (has[c]) {
        if (classes[c] >= 16) gw_update(ctx, classes[c] / 16, dj, cl[c]);
        else g_update(ctx, classes[c], dj, cl[c]);
        ++nl;
      }
    g_finalize(ctx, 1, dj, lu);
    g_solve(ctx, 1, eps, dj, ls);
    for (int c = 0; c < 6; ++c)
      if (has[c]) {
        if (classes[c] >= 16) gw_pupdate(ctx, classes[c] / 16, dj, cl[c]);
        else g_pupdate(ctx, classes[c], dj, cl[c]);
        ++nl;
      }
    nl += 4;
    std::lock_guard<std::mutex> g(mu);
    grouped_launches += nl;
  }
  if (hi > 0)
    BKTS_HIP(hipMemcpyAsync(status_host, status_dev.p, sizeof(double) * kStatusStride * hi, hipMemcpyDeviceToHost,
                            ctx->stream));
  ctx->sync();
  {
    std::lock_guard<std::mutex> g(mu);
    ++rounds;
  }
  // decisions
  for (int s = 0; s < n; ++s) {
    Job* J = jobs[s].get();
    if (!J) continue;
    const double* st = status_host + (size_t)s * kStatusStride;
    const int k = J->k;
    if (J->state == Job::FINISHING) {
      finish(s, J->final_status);
      continue;
    }
    if (J->state == Job::RESID) {
      double mx = 0.0;
      bool finite = true;
      for (int j = 0; j < k; ++j) {
        if (!std::isfinite(st[j])) finite = false;
        mx = std::max(mx, std::sqrt(std::max(st[j], 0.0)));
      }
      J->rel = J->rhs0 > 0.0 ? mx / J->rhs0 : mx;
      if (!finite) {
        J->final_status = BKTS_EBREAKDOWN;
      } else if (J->rel <= J->p.req.rtol) {
        J->final_status = BKTS_OK;
      } else if (J->outer >= (J->p.req.max_outer > 0 ? J->p.req.max_outer : 200)) {
        J->final_status = BKTS_ENOCONV;
      } else {
        ++J->outer;
        J->state = Job::INIT;
        continue;
      }
      BKTS_HIP(hipMemcpyAsync(J->p.req.y_out, J->Y.p, sizeof(double) * J->N * k, hipMemcpyDeviceToDevice,
                              ctx->stream));
      J->state = Job::FINISHING;
      continue;
    }
    if (J->state == Job::CG) {
      ++J->inner_it;
      ++J->krylov;
      const double* nrm = st + k;
      const double* nrm0 = st + 2 * k;
      const int nd = *reinterpret_cast<const int*>(st + 3 * k);
      const double tol2 = J->p.req.inner_rtol * J->p.req.inner_rtol;
      bool ok = true;
      for (int j = 0; j < k; ++j)
        if (!(nrm[j] <= tol2 * nrm0[j])) ok = false;
      const int maxit = J->p.req.max_inner > 0 ? J->p.req.max_inner : 2000;
      if (ok || nd >= k || J->inner_it >= maxit) {
        J->pending_apply = true;
        J->state = Job::RESID;
      }
    }
  }
}

void bkts_server_s::finish(int slot, int status) {
  std::unique_ptr<Job> J = std::move(jobs[slot]);
  bkts_result r{};
  r.ticket = J->p.ticket;
  r.tag = J->p.req.tag;
  r.status = status;
  r.outer_iterations = J->outer;
  r.krylov_iterations = J->krylov;
  r.rel_residual = J->rel;
  r.t_submit = J->p.t_submit;
  r.t_admit = J->t_admit;
  r.t_done = now();
  r.footprint_bytes = J->p.footprint;
  J.reset();  // frees the job's device memory (the stream is idle: the round just synchronised)
  std::lock_guard<std::mutex> g(mu);
  in_use -= r.footprint_bytes;
  --n_active;
  done.push_back(r);
  cv_done.notify_all();
  cv.notify_all();
}

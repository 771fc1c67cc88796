// Host-side internals of the bkts library: handle layouts, workspace, error plumbing and the
// launchers every translation unit shares.  Nothing here is part of the C ABI.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "../../include/bkts.h"

namespace bkts {

struct Error {
  bkts_status status;
  std::string msg;
};

std::string fmt(const char* f, ...);
void set_last_error(const std::string& m);

#define BKTS_HIP(x)                                                                              \
  do {                                                                                           \
    hipError_t e_ = (x);                                                                         \
    if (e_ != hipSuccess)                                                                        \
      throw ::bkts::Error{BKTS_EDEVICE, std::string(#x) + " failed: " + hipGetErrorString(e_)};  \
  } while (0)

#define BKTS_REQUIRE(cond, ...)                                            \
  do {                                                                     \
    if (!(cond)) throw ::bkts::Error{BKTS_EINVAL, ::bkts::fmt(__VA_ARGS__)}; \
  } while (0)

// Owning device allocation.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : p(o.p), bytes(o.bytes) { o.p = nullptr; o.bytes = 0; }
  DevBuf& operator=(DevBuf&& o) noexcept {
    release();
    p = o.p; bytes = o.bytes; o.p = nullptr; o.bytes = 0;
    return *this;
  }
  ~DevBuf() { release(); }
  void alloc(size_t n);
  void release();
  template <typename T> T* as() const { return static_cast<T*>(p); }
};

// Named scratch buffers that only grow.  A buffer's contents are undefined on return from get().
struct Workspace {
  std::map<std::string, DevBuf> bufs;
  void* get(const std::string& name, size_t bytes);
  template <typename T> T* get(const std::string& name, size_t count) {
    return static_cast<T*>(get(name, count * sizeof(T)));
  }
  size_t total_bytes() const;
};

inline size_t esize(int dtype) { return dtype == BKTS_F32 ? 4 : 8; }

// Pivot floor of the deflating k x k Gram solve in block CG (Jacobi-scaled, so a pivot is the squared
// sine of the angle between a direction and the span of the earlier ones).  FP32 Gram matrices
// carry relative noise near 1e-6 (FP32 products summed over 16-row tiles), so an FP32 pivot below
// 1e-4 is not resolved and keeping it multiplies that noise by its inverse; the stage residuals of
// a fully implicit tableau are that close to parallel.  FP64 Gram matrices resolve pivots far
// below 1e-13.
inline double cg_pivot_floor(int dtype) { return dtype == BKTS_F64 ? 1e-13 : 1e-4; }

// Resident workgroups per CU of a kernel with 256-thread workgroups (cached per kernel).
int blocks_per_cu(const void* kernel);

}  // namespace bkts

namespace bkts {
// Per-kernel device timers: HIP events recorded around each launch on the context stream, plus the
// algorithmic bytes the launch moves (the kernel's own traffic model, not hardware counters).
struct Profiler {
  struct Rec {
    int kid;
    hipEvent_t a, b;
  };
  struct Acc {
    int64_t launches = 0;
    double ms = 0.0;
    double bytes = 0.0;
    std::vector<float> samples;  // each timed launch's duration (ms), in launch order
  };
  bool enabled = false;
  int period = 1;                      // time every period-th launch of each kernel id
  int64_t seq[BKTS_K_COUNT] = {};      // launches seen per kernel id since enabling
  int open = 0;  // scopes whose end event is not recorded yet (they nest)
  // Events of the innermost scope waiting for its kernel: the next launch() carries them in its
  // dispatch packet, so their interval is that kernel's own execution (no queue gaps).
  hipEvent_t ext_a = nullptr, ext_b = nullptr;
  std::vector<hipEvent_t> pool;
  std::vector<Rec> pending;
  Acc acc[BKTS_K_COUNT];
  hipEvent_t take();
  void resolve();  // waits for pending events and folds them into acc
  void reset();
  ~Profiler();
};
}  // namespace bkts

struct bkts_ctx_s {
  int device = 0;
  hipStream_t stream = nullptr;
  int num_cu = 256;
  bkts::Workspace ws;
  double* h_pinned = nullptr;  // pinned host staging for small read-backs
  size_t h_pinned_bytes = 0;
  bkts::Profiler prof;
  bkts::DevBuf tail_counters;  // zero-initialised device words for fold+solve launches
  unsigned* tail_counter(int i);

  double* host_stage(size_t count);  // pinned buffer of at least `count` doubles
  void sync();
};

namespace bkts {
struct MgHier;  // multigrid hierarchy of an operator (mg.hip)
void mg_hier_delete(MgHier* h);
}  // namespace bkts

struct bkts_op_s {
  bkts_ctx ctx = nullptr;
  int64_t N = 0, nnz = 0;
  int format = BKTS_FMT_CSR;
  bkts_grid grid{};  // dim == 0 when the operator came from a raw CSR
  // CSR (always present)
  bkts::DevBuf rowptr, col, val, val32;
  bkts::DevBuf diag;  // K_rr (double), used for Jacobi
  bkts::DevBuf b;     // source vector (double, N), zero unless assembled with nonzero boundary data
  bool b_nonzero = false;
  // SELL-C (sigma = 1): slice s covers rows [s*C, s*C+C), width w_s, entry (row, j) at
  // sell_ptr[s] + j*C + (row - s*C); padding entries have col = row and val = 0.
  int sell_C = 64;
  int sell_uniform_w = 0;  // > 0: every slice has this width, sell_ptr[s] = s*C*w (no pointer loads needed)
  int64_t nslices = 0, sell_nnz = 0;
  // Reuse distance of the block operator in rows (a z-plane of a 3-D grid, an x-line of a 2-D
  // grid); used to schedule one strip of every period per XCD so the +-1 period neighbours stay in
  // that XCD's L2.  0 = unknown.
  int64_t strip_period = 0;
  bkts::DevBuf sell_ptr, sell_w, sell_col, sell_val, sell_val32;
  // Index-free stencil form (BKTS_FMT_STENCIL; stencil.hip): st_na > 0 distinct neighbour offsets
  // st_off[a] in rows; st_coef holds (1 + st_na) arrays of N: the diagonal, then o_a[r] = K[r, r + s_a].
  // When present, the block operator uses it instead of CSR/SELL.
  int st_na = 0;
  int64_t st_off[3] = {0, 0, 0};
  bkts::DevBuf st_coef, st_coef32;
  // Galerkin multigrid hierarchy of K and the mass (built on first use by a multigrid solve)
  mutable std::shared_ptr<bkts::MgHier> mg;
  // A Newton Jacobian (CSR on the stencil sparsity, not symmetric) keeps the stencil form of its
  // symmetric part (J + J^T) / 2 here, the operator BKTS_PREC_MG builds its hierarchy from; stale
  // once the Jacobian's values change, rebuilt on the next multigrid solve.
  mutable std::shared_ptr<bkts_op_s> mg_sym;
  mutable bool mg_sym_stale = true;
};

// Nonlinear FV operator (nonlinear.hip).
namespace bkts {

struct NlDev {
  int kind;  // 0: diffusion-reaction (mass = identity), 1: Richards (mass = theta(psi))
  int dim;
  int n[3];
  double w[3];  // 1 / h_d^2
  // diffusion-reaction
  double dc[4], rc[4];
  int bc_type[6];
  double bc_val[6];
  // Richards: van Genuchten closure, saturated conductivity per cell, z = last axis
  double tr, ts, alpha, vn, vm;
  const double* ks;
  const double* tf;  // per cell, 4 values: harm(Ks_P, Ks_Q) / h_d^2 of the face to the next cell Q along
                     // x, y, z (0 where there is none), then Ks_P
  int top_dirichlet, bottom_drain;
  double top_g, top_kr, hz;
  double lin_L;  // > 0: the mass derivative in the Jacobian is this constant (L-scheme)
};

}  // namespace bkts

struct bkts_nlop_s {
  bkts_ctx ctx = nullptr;
  bkts::NlDev nd{};
  int64_t N = 0;
  bkts_op jac = nullptr;  // stencil sparsity; values overwritten by bkts_nl_jacobian
  bkts::DevBuf ks;        // Richards: own copy of the saturated conductivity
  bkts::DevBuf tf;        // Richards: face transmissibilities and Ks per cell (NlDev::tf)
  ~bkts_nlop_s() { delete jac; }
};

struct bkts_tc_s {
  bkts_ctx ctx = nullptr;
  int k = 1;
  int m_impl = 1;       // implicit stages per step
  int explicit_first = 0;
  double tau = 1.0;
  std::vector<double> Ai;  // m_impl x m_impl implicit part of the tableau
  std::vector<double> ae;  // couplings of implicit stages to the eliminated explicit stage
  std::vector<double> ci;
  // window matrices for each phase, row-major k x k
  std::vector<std::vector<double>> A1, A2;
  // fully implicit tableau (an implicit stage couples to a later one): windows hold whole steps,
  // the front is always stage 0, and the splitting uses the averaged coefficient beta_avg
  int fully_implicit = 0;
  double beta_avg = 0.0;
};

// Splitting coefficient beta of J = M/tau + beta K for a window whose front is implicit stage
// `phase`: the front stage's diagonal entry, or the averaged coefficient of a fully implicit tableau.
inline double tc_beta(const bkts_tc_s& t, int phase) { return t.fully_implicit ? t.beta_avg : t.A2[phase][0]; }

namespace bkts {

// RAII timer around the launches of one kernel (no-op unless profiling is enabled).
// Times one kernel category.  The scope's interval is the execution of the next kernel started
// with launch() (timestamps of that dispatch); if no kernel is launched before end(), the
// interval is empty.
struct ProfScope {
  bkts_ctx ctx;
  int kid;
  hipEvent_t a = nullptr, b = nullptr;
  ProfScope(bkts_ctx c, int k, double bytes);
  void end();
  ~ProfScope() { end(); }
};

// Launch on the context stream; a pending ProfScope's events travel with this dispatch.
template <typename F, typename... Args>
inline void launch(bkts_ctx ctx, F kernel, dim3 grid, dim3 block, uint32_t shmem, Args... args) {
  Profiler& p = ctx->prof;
  hipEvent_t ea = p.ext_a, eb = p.ext_b;
  if (ea) {
    p.ext_a = p.ext_b = nullptr;
    p.open -= 1;
  }
  hipExtLaunchKernelGGL(kernel, grid, block, shmem, ctx->stream, ea, eb, 0, args...);
}

// ---- operator building (op.hip)
void op_build_sell(bkts_op op);
// dinv[r] = 1 / (a + b K_rr): inverse diagonal of a I + b K (Jacobi preconditioner)
void jacobi_inverse(bkts_ctx ctx, const bkts_op_s& op, double a, double b, double* dinv);
void op_finish(bkts_op op);  // diag, fp32 copies, SELL if requested
void op_refresh_values(bkts_op op);  // after CSR values changed: diag, SELL values, FP32 copies
// Index-free stencil form from the CSR (stencil.hip); BKTS_EINVAL unless K is a symmetric operator
// whose entries all lie at the grid-neighbour offsets.
void op_build_stencil(bkts_op op);
void spmm_stencil(bkts_ctx ctx, const bkts_op_s& op, int dtype, int k, double cb, const void* B, int ldb,
                  double alpha, const void* X, int ldx, double beta, void* Y, int ldy);
// Block-CG reductions folded into the finest prolongation of a V-cycle Z = V(R) (k in {1, 2, 4}):
// in: Q (N x k, contiguous, the V-cycle's dtype); out: partials of gamma = R^T Z, T = Q^T Z and
// nrm = diag(R^T R), laid out [gamma (k*k) | T (k*k) | nrm (k)] x nslots (workspace owned by the
// context).  nslots == 0 on return: the hierarchy is too small for a separate finest prolongation and
// nothing was reduced.
struct MgFuse {
  const void* Q = nullptr;
  double* partials = nullptr;
  int64_t nslots = 0;
};
// Z = V-cycle(F) for a I + b K (mg.hip): symmetric geometric multigrid on the stencil form, N x k
// contiguous blocks of type dtype.  BKTS_EINVAL without the stencil form.
void mg_vcycle(bkts_ctx ctx, const bkts_op_s& op, int dtype, int k, double a, double b, const void* F, void* Z,
               MgFuse* fuse = nullptr);
// Whether a V-cycle of width k on this operator has a separate finest prolongation that can fold the
// block-CG reductions (builds the hierarchy on first use).
bool mg_fusable(bkts_ctx ctx, const bkts_op_s& op, int k);
// Recompute the hierarchy of an operator whose stencil values changed (no-op before its first use).
void mg_refresh(bkts_ctx ctx, const bkts_op_s& op);
// The operator a multigrid preconditioner for `op` is built from: op itself in the stencil form,
// the stencil form of the symmetric part of a Newton Jacobian (refreshed when stale), else null.
const bkts_op_s* mg_source(bkts_ctx ctx, const bkts_op_s& op);
// The empty stencil-form holder of the symmetric part of J (grid operators only, else null), and its
// refresh from J's current CSR values: diagonal J_rr, couplings (J[r, r+s] + J[r+s, r]) / 2.
std::shared_ptr<bkts_op_s> sym_stencil_create(const bkts_op_s& J);
void sym_stencil_refresh(bkts_ctx ctx, const bkts_op_s& J, bkts_op_s& S);

// ---- nonlinear operator (nonlinear.hip)
bkts_nlop nlop_create(bkts_ctx ctx, const bkts_grid* grid, const bkts_nl_coeffs* c);
// F[:, j] = f(Y[:, j]) for j < k
void nl_eval(bkts_ctx ctx, const bkts_nlop_s& nl, int k, const double* Y, int ldy, double* F, int ldf);
// Mass term of the semi-discrete problem, column-wise: M[:, j] = m(Y[:, j]) (identity or theta)
void nl_mass(bkts_ctx ctx, const bkts_nlop_s& nl, int k, const double* Y, int ldy, double* M, int ldm);
bkts_nlop richards_create(bkts_ctx ctx, const bkts_grid* grid, const double* ks, const bkts_richards_params* p);
// nl.jac values = alpha I + beta Df(u) (u: column with stride ldu)
void nl_jacobian(bkts_ctx ctx, bkts_nlop_s& nl, const double* u, int ldu, double alpha, double beta);
// R = Y A1^T + F(Y) A2^T - B0 with column norms (A1, A2 device, row-major, physical order)
void nl_residual(bkts_ctx ctx, const bkts_nlop_s& nl, int k, const double* Y, int ldy, const double* A1,
                 const double* A2, const double* B0, int ldb0, int nb0, const int* b0_to_col, double* R, int ldr,
                 double* nrm);

// ---- kernels (launchers). All enqueue on ctx->stream.
// Y = cb*B + alpha*X + beta*K X   (B may be null). dtype F64/F32 for X, Y, B.
void spmm(bkts_ctx ctx, const bkts_op_s& op, int dtype, int k, double cb, const void* B, int ldb,
          double alpha, const void* X, int ldx, double beta, void* Y, int ldy);

// G = X^T Y with the partials in the library's fixed per-device scratch array (no allocation);
// scratch_init(device) records that device's address of the array (device current, once).
void gram_noalloc(bkts_ctx ctx, int dtype, int64_t N, int k, const void* X, int ldx, const void* Y, int ldy,
                  double* G);
void scratch_init(int device);

// Reductions produce per-block partials that finalize_partials() folds, in a fixed order.
int reduce_blocks(bkts_ctx ctx, int64_t N, int k);
void finalize_partials(bkts_ctx ctx, const double* partials, int nblocks, int nentries, double* out);
// k x k result from partials laid out as entry (a*KP + b) x nblocks
void finalize_gram(bkts_ctx ctx, const double* partials, int nblocks, int k, int KP, double* out);
// Up to three folds in one launch: set i is a k x k Gram (vector == 0) or a k-vector (vector == 1).
struct FoldSet {
  const double* partials;
  int KP;
  int vector;
  double* out;
};
void finalize_sets(bkts_ctx ctx, int nblocks, int k, const FoldSet* sets, int nsets);

// Coefficient step after a block-CG kernel in ONE launch: fold the kernel's partials in a fixed
// order (one workgroup per entry) and let the last workgroup solve the k x k system.  After the SpMM: G and alpha = G^+ gamma_in
// (and the deflation count).  After the update: gamma, T, nrm and beta = -G^+ T.
struct CgTail {
  unsigned* counter = nullptr;  // device word, zero between launches
  double eps = 0.0;
  double* G = nullptr;
  const double* gamma_in = nullptr;
  double* alpha = nullptr;
  int* ndefl = nullptr;
  double* gamma = nullptr;
  double* T = nullptr;
  double* nrm = nullptr;
  double* beta = nullptr;
  // mode 1, optional: device-visible pinned host memory that the solving workgroup fills with
  // nrm[0..k) followed by *ndefl (as an int), so the host reads the norms without a copy launch
  double* host = nullptr;
};

// fold.hip: mode 0 after a Gram kernel, mode 1 after an update kernel; kp in {1, 2, 4, 16, 32}.
void fold_solve(bkts_ctx ctx, int mode, int kp, int k, const double* partials, int64_t nslots, const CgTail& t);

// Row-per-thread block kernels for k in {1, 2, 4} (rowk.hip); contiguous blocks (ld = k).
bool rk_eligible(int k);
void rk_spmm_gram(bkts_ctx ctx, const bkts_op_s& op, int dtype, int k, double alpha, const void* P, double beta,
                  void* Q, double* G, const CgTail* tail = nullptr);  // Q = alpha P + beta K P, G = P^T Q
void rk_cg_update(bkts_ctx ctx, int dtype, int64_t N, int k, void* X, const void* P, void* R, const void* Q,
                  const double* alpha, const double* dinv, double* gamma, double* Tm, double* nrm,
                  const CgTail* tail = nullptr);
void rk_cg_pupdate(bkts_ctx ctx, int dtype, int64_t N, int k, void* P, const void* R, const double* beta,
                   const double* dinv);
// X += P alpha, R -= Q alpha with no reductions (the multigrid prolongation folds them instead)
void rk_cg_xr_update(bkts_ctx ctx, int dtype, int64_t N, int k, void* X, const void* P, void* R, const void* Q,
                     const double* alpha);
// The two halves on their own: R -= Q alpha, and X += P alpha
void rk_cg_r_update(bkts_ctx ctx, int dtype, int64_t N, int k, void* R, const void* Q, const double* alpha);
void rk_cg_x_update(bkts_ctx ctx, int dtype, int64_t N, int k, void* X, const void* P, const double* alpha);
// X += P alpha and P = Z + P beta in one pass (both read the old P); x_init: X = P alpha (X not read)
void rk_cg_xp_update(bkts_ctx ctx, int dtype, int64_t N, int k, void* X, void* P, const void* Z, const double* alpha,
                     const double* beta, bool x_init = false);
void rk_gram(bkts_ctx ctx, int dtype, int64_t N, int k, const void* X, const void* Y, double* G);
// G1 = X1^T Y and G2 = X2^T Y in one pass (k in {1, 2, 4}, contiguous blocks)
void rk_gram2(bkts_ctx ctx, int dtype, int64_t N, int k, const void* X1, const void* X2, const void* Y, double* G1,
              double* G2);
void rk_rmul(bkts_ctx ctx, int dtype, int64_t N, int k, const void* X, const double* C, double c0, double c1,
             void* Y);

// MFMA-based block kernels for 8 <= k <= 32 (mfma.hip); contiguous blocks (ld = k) unless noted.
bool mf_eligible(int k);
// Block Gram-Schmidt against nblk <= mf_mgs_max_blocks(k) blocks V_i = V0 + i * vstride (elements):
// mf_mgram writes per-slot partials of every V_i^T W (nslots_out slots; the partial buffer holds
// nblk * KP^2 * mf_mgram_slots() doubles, KP = 16 or 32); mf_mgs_finalize sums them into C (nblk
// row-major k x k blocks) and stores or adds them into H at (r0 + i k, c0) (KP = 1 for k = 1, the
// mdot partials); mf_mrmul applies W -= sum_i V_i C_i.
int mf_mgs_max_blocks(int k);
int64_t mf_mgram_slots(bkts_ctx ctx, int dtype, int64_t N, int k);
void mf_mgram(bkts_ctx ctx, int dtype, int64_t N, int k, int nblk, const void* V0, int64_t vstride, const void* W,
              double* partials_out, int* nslots_out);
void mf_mgs_finalize(bkts_ctx ctx, const double* partials, int nslots, int k, int nblk, double* C, double* H, int ldh,
                     int r0, int c0, bool accumulate);
void mf_mrmul(bkts_ctx ctx, int dtype, int64_t N, int k, int nblk, const void* V0, int64_t vstride, const double* C,
              void* W);
// The same for single columns (k = 1, any length n): nblk <= mdot_max_blocks() dot products
// (partials: nblk * mdot_slots() doubles; finalize with mf_mgs_finalize and k = 1) and the update.
int mdot_max_blocks();
int64_t mdot_slots(bkts_ctx ctx, int64_t n);
void mdot(bkts_ctx ctx, int dtype, int64_t n, int nblk, const void* V0, int64_t vstride, const void* W,
          double* partials_out, int* nslots_out);
void maxpy(bkts_ctx ctx, int dtype, int64_t n, int nblk, const void* V0, int64_t vstride, const double* C, void* W);
void mf_gram(bkts_ctx ctx, int dtype, int64_t N, int k, const void* X, int ldx, const void* Y, int ldy, double* G);
void mf_spmm_gram(bkts_ctx ctx, const bkts_op_s& op, int dtype, int k, double alpha, const void* P, double beta,
                  void* Q, double* G);  // Q = alpha P + beta K P, G = P^T Q
void mf_cg_update(bkts_ctx ctx, int dtype, int64_t N, int k, void* X, const void* P, void* R, const void* Q,
                  const double* alpha, const double* dinv, double* gamma,
                  double* Tm, double* nrm);
void mf_cg_pupdate(bkts_ctx ctx, int dtype, int64_t N, int k, void* P, const void* R, const double* beta,
                   const double* dinv);
void mf_rmul(bkts_ctx ctx, int dtype, int64_t N, int k, const void* X, const double* C, double c0, double c1,
             void* Y);

// G = X^T Y (device, k x k row-major)
void gram(bkts_ctx ctx, int dtype, int64_t N, int k, const void* X, int ldx, const void* Y, int ldy,
          double* G);

// Column-wise dot products of npairs (1..3) pairs of contiguous N x k blocks: out[p][j] =
// sum_r X_p[r, j] Y_p[r, j] (FP64 accumulation, fixed-order reduction; out[p] device, k values).
void col_dots(bkts_ctx ctx, int dtype, int64_t N, int k, int npairs, const void* const* X, const void* const* Y,
              double* const* out);
// Column sums of squares: out[j] = sum_r X[r, j]^2 (device, k)
void colnorms2(bkts_ctx ctx, int dtype, int64_t N, int k, const void* X, int ldx, double* out);

// Block CG update (all blocks N x k, same dtype, ld = k):
//   X += P*alpha ; R -= Q*alpha ; Z = Dinv R ;  gamma = R^T Z ; T = Q^T Z ; nrm[j] = ||R_j||^2
// alpha (k x k) read from device memory; outputs gamma, T, nrm in device memory.
void cg_update(bkts_ctx ctx, int dtype, int64_t N, int k, void* X, const void* P, void* R, const void* Q,
               const double* alpha_dev, const double* dinv,
               double* gamma, double* T, double* nrm);
// P = Dinv R + P*beta
void cg_pupdate(bkts_ctx ctx, int dtype, int64_t N, int k, void* P, const void* R, const double* beta_dev,
                const double* dinv);

// General right-multiply-accumulate: Y = c0*Y + c1*X*C  (C: device k x k, row-major)
void block_rmul(bkts_ctx ctx, int dtype, int64_t N, int k, const void* X, int ldx, const double* C,
                double c0, double c1, void* Y, int ldy);

// block_cast_scale between FP64 and FP32 for contiguous 16-byte aligned blocks of k in {1, 2, 4}
// columns, one row per thread; returns false (and does nothing) for any other shape.
bool rk_cast(bkts_ctx ctx, int64_t N, int k, int src_t, const void* src, int dst_t, void* dst, const double* s,
             bool invert, bool accumulate, bool norm2, double coef);

// Scaled casts: dst = coef * src * diag(s) (s device, k; null = ones), between F64 and F32 blocks;
// invert_s divides by s; norm2: s holds squared column norms and column c scales by sqrt(s[c]) (1
// for a zero column); accumulate adds into dst.
void block_cast_scale(bkts_ctx ctx, int64_t N, int k, int src_t, const void* src, int lds, int dst_t,
                      void* dst, int ldd, const double* s, bool invert_s, bool accumulate, bool norm2 = false,
                      double coef = 1.0);

// All-at-once residual (fused).  A1t, A2t: device k x k transposed window matrices (A^T, row-major).
// b0cols: host list of (b0 column index -> R column index).
void residual(bkts_ctx ctx, const bkts_op_s& op, int k, const double* Y, int ldy, const double* A1t,
              const double* A2t, const double* b_rowsum, const double* B0, int ldb0, int nb0,
              const int* b0_to_col, double* R, int ldr, double* nrm);

// Single-workgroup kernels for block GMRES / BiCGStab (small2.hip).
void small_cholqr(bkts_ctx ctx, int k, const double* G, double eps, double* Rinv, double* R, int* ndefl);
void small_gemm(bkts_ctx ctx, int k, const double* A, const double* B, double alpha, double* C);
void small_lu_solve2(bkts_ctx ctx, int k, const double* M, const double* B1, double s1, double* X1, const double* B2,
                     double s2, double* X2, double eps);
void small_omega(bkts_ctx ctx, int k, const double* TS, const double* TT, double* out);
// out = diag(sign * a_j / b_j) as a k x k matrix, for device k-vectors a, b (0 where b_j is zero or
// the ratio is not finite)
void small_diag_ratio(bkts_ctx ctx, int k, const double* a, const double* b, double sign, double* out);
// Largest Hessenberg row count (m + 1)k that block GMRES may use for block width k.
int gmres_max_rows(int k);
// Incremental Householder QR of block column jb of the block Hessenberg matrix (rows (jb+2)k of H,
// column-major with leading dimension ldh), with the triangular factor Rq, reflectors Vr (2k per
// column), Br, and Gq = Q^T [S; 0] ((m+1)k x k row-major) kept between calls; resn = per-column
// least-squares residual norms.
void gmres_qr_step(bkts_ctx ctx, int k, int jb, const double* H, int ldh, const double* S, double* Rq, double* Vr,
                   double* Br, double* Gq, double* resn);
// Y (nc x k row-major) = R^-1 Gq over the first nc rows, dropping |R_ii| <= eps max|R_jj|.
void gmres_backsolve(bkts_ctx ctx, int k, int nc, const double* Rq, int ldh, const double* Gq, double eps, double* Y);

// k x k dense kernels on one workgroup (small.hip).
// alpha = G^+ S with truncated Cholesky of the Jacobi-scaled G (threshold `eps`); writes
// ndefl (device int) = number of deflated directions.  sign = +1 or -1 multiplies the result.
void small_spd_solve(bkts_ctx ctx, int k, const double* G, const double* S, double sign, double eps,
                     double* out, int* ndefl);

}  // namespace bkts

// Nonlinear FV operators for the Newton form of Algorithm 1 (Sec. 2.2): the column-wise f, the
// mass term m (identity, or theta for Richards' equation, Sec. 4.3), the exact Jacobian
// alpha m'(u) + beta Df(u) assembled on the fixed stencil sparsity, and the fused window residual
// R = m(Y) A1^T + F(Y) A2^T - B0 (F_j = f(Y_j)).
//
// Diffusion-reaction, f(u) = -div_h(D(u) grad_h u) - r(u) (cell-centred, per unit volume): interior
// face P|Q along axis d contributes (D(u_P) + D(u_Q))/2 * (u_P - u_Q) / h_d^2; a Dirichlet face
// with value g contributes (D(u_P) + D(g))/2 * 2 (u_P - g) / h_d^2; zero-flux faces nothing.
//
// Richards, f(psi) = -div_h(K(psi) grad_h(psi + z)) with z the last axis: interior face
// harm(Ks_P, Ks_Q) (kr_P + kr_Q)/2 (H_P - H_Q) / h_d^2 with H = psi + z; a Dirichlet top face
// 2 Ks_P (kr_P + kr(g))/2 (H_P - (g + 1)) / h^2; a free-drainage bottom face Ks_P kr_P / h.
#include <cmath>

#include "devcommon.hpp"
#include "internal.hpp"

namespace bkts {
namespace {

using dev::TileGeom;

__device__ __forceinline__ double poly(const double (&c)[4], double u) { return ((c[3] * u + c[2]) * u + c[1]) * u + c[0]; }
__device__ __forceinline__ double dpoly(const double (&c)[4], double u) { return (3.0 * c[3] * u + 2.0 * c[2]) * u + c[1]; }

// Grid coordinates of cell r (32-bit arithmetic: operators are created with N < 2^31).
__device__ __forceinline__ void coords(const NlDev& g, int64_t r, int (&i)[3]) {
  uint32_t q = (uint32_t)r;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    if (d < g.dim) {
      const uint32_t q2 = q / (uint32_t)g.n[d];
      i[d] = (int)(q - q2 * (uint32_t)g.n[d]);
      q = q2;
    } else {
      i[d] = 0;
    }
  }
}

__device__ __forceinline__ int64_t stride_of(const NlDev& g, int d) {
  int64_t s = 1;
  for (int e = 0; e < d; ++e) s *= g.n[e];
  return s;
}

// ---- van Genuchten closure (eq. RelationshipsThetaK), s = theta / theta_s as printed
__device__ __forceinline__ double vg_se(const NlDev& g, double psi) {
  return psi < 0.0 ? pow(1.0 + pow(-g.alpha * psi, g.vn), -g.vm) : 1.0;
}
__device__ __forceinline__ double vg_dse(const NlDev& g, double psi) {
  if (!(psi < 0.0)) return 0.0;
  const double a = -g.alpha * psi;
  return g.vm * g.vn * g.alpha * pow(a, g.vn - 1.0) * pow(1.0 + pow(a, g.vn), -g.vm - 1.0);
}
__device__ __forceinline__ double vg_theta(const NlDev& g, double psi) { return g.tr + (g.ts - g.tr) * vg_se(g, psi); }
__device__ __forceinline__ double vg_dtheta(const NlDev& g, double psi) { return (g.ts - g.tr) * vg_dse(g, psi); }
__device__ __forceinline__ double vg_kr(const NlDev& g, double psi) {
  const double s = vg_theta(g, psi) / g.ts;
  const double gg = 1.0 - pow(1.0 - pow(s, 1.0 / g.vm), g.vm);
  return sqrt(s) * gg * gg;
}
__device__ __forceinline__ double vg_dkr(const NlDev& g, double psi) {
  const double s = vg_theta(g, psi) / g.ts;
  const double ds = vg_dtheta(g, psi) / g.ts;
  const double w = 1.0 - pow(s, 1.0 / g.vm);
  const double gg = 1.0 - pow(w, g.vm);
  const double dg = w > 0.0 ? pow(w, g.vm - 1.0) * pow(s, 1.0 / g.vm - 1.0) : 0.0;
  return (0.5 / sqrt(s) * gg * gg + sqrt(s) * 2.0 * gg * dg) * ds;
}

// theta(psi) and kr(psi) together: one saturation evaluation serves both (same operations as
// vg_theta and vg_kr, so the same values)
__device__ __forceinline__ void vg_theta_kr(const NlDev& g, double psi, double& theta, double& kr) {
  theta = vg_theta(g, psi);
  const double s = theta / g.ts;
  const double gg = 1.0 - pow(1.0 - pow(s, 1.0 / g.vm), g.vm);
  kr = sqrt(s) * gg * gg;
}

__device__ __forceinline__ double mass_at(const NlDev& g, double u) { return g.kind == 1 ? vg_theta(g, u) : u; }

__device__ __forceinline__ double harm(double a, double b) { return a + b > 0.0 ? 2.0 * a * b / (a + b) : 0.0; }

// Richards f(psi)_r for the column of u with stride ld
__device__ double ri_f_at(const NlDev& g, const double* u, int ld, int64_t r) {
  int i[3];
  coords(g, r, i);
  const int zd = g.dim - 1;
  const double up = u[r * ld], krp = vg_kr(g, up), ksp = g.ks[r];
  const double zp = (i[zd] + 0.5) * g.hz, Hp = up + zp;
  double f = 0.0;
  for (int d = 0; d < g.dim; ++d) {
    const int64_t st = stride_of(g, d);
    for (int side = 0; side < 2; ++side) {
      const bool interior = side == 0 ? i[d] > 0 : i[d] < g.n[d] - 1;
      if (interior) {
        const int64_t q = side == 0 ? r - st : r + st;
        const double uq = u[q * ld];
        const double Hq = uq + (d == zd ? zp + (side == 0 ? -g.hz : g.hz) : zp);
        f += harm(ksp, g.ks[q]) * g.w[d] * 0.5 * (krp + vg_kr(g, uq)) * (Hp - Hq);
      } else if (d == zd && side == 1 && g.top_dirichlet) {
        f += 2.0 * ksp * 0.5 * (krp + g.top_kr) * (Hp - (g.top_g + 1.0)) * g.w[d];
      } else if (d == zd && side == 0 && g.bottom_drain) {
        f += ksp * krp / g.hz;
      }
    }
  }
  return f;
}

// Richards f(psi)_r as ri_f_at, with kr read from kr[q * ldk] (evaluated once per cell beforehand)
// instead of evaluated at the cell and at each neighbour.
__device__ double ri_f_cached(const NlDev& g, const double* u, int ld, const double* kr, int ldk, int64_t r) {
  int i[3];
  coords(g, r, i);
  const int zd = g.dim - 1;
  const double up = u[r * ld], krp = kr[r * ldk], ksp = g.ks[r];
  const double zp = (i[zd] + 0.5) * g.hz, Hp = up + zp;
  double f = 0.0;
  int64_t st = 1;
  for (int d = 0; d < g.dim; ++d) {
    for (int side = 0; side < 2; ++side) {
      const bool interior = side == 0 ? i[d] > 0 : i[d] < g.n[d] - 1;
      if (interior) {
        const int64_t q = side == 0 ? r - st : r + st;
        const double uq = u[q * ld];
        const double Hq = uq + (d == zd ? zp + (side == 0 ? -g.hz : g.hz) : zp);
        f += harm(ksp, g.ks[q]) * g.w[d] * 0.5 * (krp + kr[q * ldk]) * (Hp - Hq);
      } else if (d == zd && side == 1 && g.top_dirichlet) {
        f += 2.0 * ksp * 0.5 * (krp + g.top_kr) * (Hp - (g.top_g + 1.0)) * g.w[d];
      } else if (d == zd && side == 0 && g.bottom_drain) {
        f += ksp * krp / g.hz;
      }
    }
    st *= g.n[d];
  }
  return f;
}

// theta and kr of every entry of the first k columns of Y, into TH and KR (N x k, contiguous)
__global__ void ri_cache_kernel(NlDev g, int64_t N, int k, const double* Y, int ldy, double* TH, double* KR) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N * k) return;
  const int64_t r = i / k;
  const int c = (int)(i - r * k);
  double th, kr;
  vg_theta_kr(g, Y[r * ldy + c], th, kr);
  TH[i] = th;
  KR[i] = kr;
}

// f(u)_r for the column of u with stride ld (u[q * ld])
__device__ double f_at(const NlDev& g, const double* u, int ld, int64_t r) {
  if (g.kind == 1) return ri_f_at(g, u, ld, r);
  int i[3];
  coords(g, r, i);
  const double up = u[r * ld];
  const double Dp = poly(g.dc, up);
  double f = -poly(g.rc, up);
  for (int d = 0; d < g.dim; ++d) {
    const int64_t st = stride_of(g, d);
    for (int side = 0; side < 2; ++side) {
      const bool interior = side == 0 ? i[d] > 0 : i[d] < g.n[d] - 1;
      if (interior) {
        const double uq = u[(side == 0 ? r - st : r + st) * ld];
        f += 0.5 * (Dp + poly(g.dc, uq)) * (up - uq) * g.w[d];
      } else if (g.bc_type[2 * d + side] == BKTS_BC_DIRICHLET) {
        const double gv = g.bc_val[2 * d + side];
        f += 0.5 * (Dp + poly(g.dc, gv)) * (up - gv) * 2.0 * g.w[d];
      }
    }
  }
  return f;
}

__global__ void nl_eval_kernel(NlDev g, int64_t N, int k, const double* Y, int ldy, double* F, int ldf) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N * k) return;
  const int64_t r = i / k;
  const int c = (int)(i % k);
  F[r * ldf + c] = f_at(g, Y + c, ldy, r);
}

__global__ void nl_mass_kernel(NlDev g, int64_t N, int k, const double* Y, int ldy, double* M, int ldm) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N * k) return;
  const int64_t r = i / k;
  const int c = (int)(i % k);
  M[r * ldm + c] = mass_at(g, Y[r * ldy + c]);
}

// Row r of the Richards Jacobian alpha m'(u) + beta Df(u) (m' = theta' or lin_L).
__device__ void ri_jac_row(const NlDev& g, const double* u, int ldu, int64_t r, double alpha, double beta,
                           double& diag, double (&off)[6], bool (&has)[6]) {
  int i[3];
  coords(g, r, i);
  const int zd = g.dim - 1;
  const double up = u[r * ldu], krp = vg_kr(g, up), dkrp = vg_dkr(g, up), ksp = g.ks[r];
  const double zp = (i[zd] + 0.5) * g.hz, Hp = up + zp;
  double dd = 0.0;
  for (int f = 0; f < 6; ++f) has[f] = false;
  for (int d = 0; d < g.dim; ++d) {
    const int64_t st = stride_of(g, d);
    for (int side = 0; side < 2; ++side) {
      const int f = 2 * d + side;
      const bool interior = side == 0 ? i[d] > 0 : i[d] < g.n[d] - 1;
      if (interior) {
        const int64_t q = side == 0 ? r - st : r + st;
        const double uq = u[q * ldu];
        const double Hq = uq + (d == zd ? zp + (side == 0 ? -g.hz : g.hz) : zp);
        const double wk = harm(ksp, g.ks[q]) * g.w[d];
        const double m = 0.5 * (krp + vg_kr(g, uq)), dH = Hp - Hq;
        dd += wk * (m + 0.5 * dkrp * dH);
        off[f] = beta * wk * (-m + 0.5 * vg_dkr(g, uq) * dH);
        has[f] = true;
      } else if (d == zd && side == 1 && g.top_dirichlet) {
        dd += 2.0 * ksp * (0.5 * (krp + g.top_kr) + 0.5 * dkrp * (Hp - (g.top_g + 1.0))) * g.w[d];
      } else if (d == zd && side == 0 && g.bottom_drain) {
        dd += ksp * dkrp / g.hz;
      }
    }
  }
  const double mp = g.lin_L > 0.0 ? g.lin_L : vg_dtheta(g, up);
  diag = alpha * mp + beta * dd;
}

// Row r of J = alpha m'(u) + beta Df(u), written in the stencil's sorted column order
// (z-, y-, x-, diagonal, x+, y+, z+) starting at val[rowptr[r]].
__global__ void nl_jac_kernel(NlDev g, int64_t N, const double* u, int ldu, double alpha, double beta,
                              const int32_t* rowptr, double* val) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= N) return;
  if (g.kind == 1) {
    double diag, off[6];
    bool has[6];
    ri_jac_row(g, u, ldu, r, alpha, beta, diag, off, has);
    int64_t p = rowptr[r];
    for (int d = g.dim - 1; d >= 0; --d)
      if (has[2 * d]) val[p++] = off[2 * d];
    val[p++] = diag;
    for (int d = 0; d < g.dim; ++d)
      if (has[2 * d + 1]) val[p++] = off[2 * d + 1];
    return;
  }
  int i[3];
  coords(g, r, i);
  const double up = u[r * ldu];
  const double Dp = poly(g.dc, up), dDp = dpoly(g.dc, up);
  double diag = -dpoly(g.rc, up);
  double off[6];
  bool has[6];
  for (int f = 0; f < 6; ++f) has[f] = false;
  for (int d = 0; d < g.dim; ++d) {
    const int64_t st = stride_of(g, d);
    for (int side = 0; side < 2; ++side) {
      const int f = 2 * d + side;
      const bool interior = side == 0 ? i[d] > 0 : i[d] < g.n[d] - 1;
      if (interior) {
        const double uq = u[(side == 0 ? r - st : r + st) * ldu];
        const double Dq = poly(g.dc, uq), dDq = dpoly(g.dc, uq);
        const double Df = 0.5 * (Dp + Dq), diff = up - uq;
        diag += (Df + 0.5 * dDp * diff) * g.w[d];
        off[f] = (-Df + 0.5 * dDq * diff) * g.w[d];
        has[f] = true;
      } else if (g.bc_type[f] == BKTS_BC_DIRICHLET) {
        const double gv = g.bc_val[f];
        diag += (0.5 * (Dp + poly(g.dc, gv)) + 0.5 * dDp * (up - gv)) * 2.0 * g.w[d];
      }
    }
  }
  int64_t p = rowptr[r];
  for (int d = g.dim - 1; d >= 0; --d)
    if (has[2 * d]) val[p++] = beta * off[2 * d];
  val[p++] = alpha + beta * diag;
  for (int d = 0; d < g.dim; ++d)
    if (has[2 * d + 1]) val[p++] = beta * off[2 * d + 1];
}

struct NlResArgs {
  NlDev g;
  int64_t N;
  int k;
  const double* Y;
  int ldy;
  const double* A1;
  const double* A2;
  const double* B0;
  int ldb0, nb0;
  int b0col[8];
  double* R;
  int ldr;
  double* partials;
  int64_t tps;
  const double* th;  // Richards: theta and kr of every entry (N x k), or null
  const double* kr;
};

template <int KP>
constexpr int nlres_lds() {
  return (2 * TileGeom<KP>::LDS_DOUBLES > 4 * KP) ? 2 * TileGeom<KP>::LDS_DOUBLES : 4 * KP;
}

template <int KP>
__global__ __launch_bounds__(256) void nl_residual_kernel(NlResArgs a) {
  using G = TileGeom<KP>;
  __shared__ __align__(16) double lds[nlres_lds<KP>()];
  double* Yl = lds;
  double* Fl = lds + G::LDS_DOUBLES;
  const int t = threadIdx.x, c = t % KP, r0 = t / KP;
  const int64_t slot = dev::xcd_slot(blockIdx.x, gridDim.x);
  const int64_t ntiles = (a.N + G::RT - 1) / G::RT;
  const bool cok = c < a.k;
  double a1[KP], a2[KP];
#pragma unroll
  for (int j = 0; j < KP; ++j) {
    a1[j] = (cok && j < a.k) ? a.A1[c * a.k + j] : 0.0;
    a2[j] = (cok && j < a.k) ? a.A2[c * a.k + j] : 0.0;
  }
  int b0j = -1;
  for (int j = 0; j < a.nb0; ++j)
    if (a.b0col[j] == c) b0j = j;
  double nacc[1] = {0.0};
  const int64_t tend = (slot + 1) * a.tps < ntiles ? (slot + 1) * a.tps : ntiles;
  for (int64_t tile = slot * a.tps; tile < tend; ++tile) {
    const int64_t row0 = tile * G::RT;
    for (int i = 0; i < G::RPT; ++i) {
      const int row = r0 + i * G::RS;
      const int64_t gr = row0 + row;
      const bool ok = gr < a.N && cok;
      if (a.kr) {
        Yl[row * G::LDL + c] = ok ? a.th[gr * a.k + c] : 0.0;
        Fl[row * G::LDL + c] = ok ? ri_f_cached(a.g, a.Y + c, a.ldy, a.kr + c, a.k, gr) : 0.0;
      } else {
        Yl[row * G::LDL + c] = ok ? mass_at(a.g, a.Y[gr * a.ldy + c]) : 0.0;
        Fl[row * G::LDL + c] = ok ? f_at(a.g, a.Y + c, a.ldy, gr) : 0.0;
      }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < G::RPT; ++i) {
      const int row = r0 + i * G::RS;
      const int64_t gr = row0 + row;
      if (gr < a.N && cok) {
        double r = dev::lds_row_dot<KP>(Yl, row, a1) + dev::lds_row_dot<KP>(Fl, row, a2);
        if (b0j >= 0) r -= a.B0[gr * a.ldb0 + b0j];
        a.R[gr * a.ldr + c] = r;
        nacc[0] = fma(r, r, nacc[0]);
      }
    }
    __syncthreads();
  }
  dev::block_reduce_store<KP, 1>(nacc, lds, a.partials, gridDim.x, slot);
}

template <int KP>
void launch_nlres(bkts_ctx ctx, NlResArgs a, double* nrm) {
  using G = TileGeom<KP>;
  const int64_t ntiles = (a.N + G::RT - 1) / G::RT;
  const int64_t cap = 2 * (int64_t)ctx->num_cu;
  int64_t ns = ntiles < cap ? ntiles : cap;
  if (ns < 1) ns = 1;
  a.tps = (ntiles + ns - 1) / ns;
  a.partials = ctx->ws.get<double>("nlres_partials", (size_t)KP * ns);
  ProfScope prof(ctx, BKTS_K_RESIDUAL, 16.0 * a.N * a.k + 8.0 * a.N * a.nb0);
  launch(ctx, (nl_residual_kernel<KP>), dim3(ns), dim3(256), 0, a);
  BKTS_HIP(hipGetLastError());
  prof.end();
  finalize_partials(ctx, a.partials, (int)ns, a.k, nrm);
}

}  // namespace

bkts_op fv_assemble(bkts_ctx ctx, const bkts_grid* grid, const bkts_fv_coeffs* c, int format);

bkts_nlop nlop_create(bkts_ctx ctx, const bkts_grid* grid, const bkts_nl_coeffs* c) {
  BKTS_REQUIRE(grid && c, "grid and coeffs must not be NULL");
  BKTS_REQUIRE(grid->dim >= 1 && grid->dim <= 3, "grid dim must be 1, 2 or 3");
  auto* nl = new bkts_nlop_s();
  try {
    nl->ctx = ctx;
    NlDev& g = nl->nd;
    g.kind = 0;
    g.dim = grid->dim;
    nl->N = 1;
    for (int d = 0; d < 3; ++d) {
      g.n[d] = d < grid->dim ? grid->n[d] : 1;
      BKTS_REQUIRE(g.n[d] >= 1, "grid n[%d] must be >= 1", d);
      g.w[d] = (double)g.n[d] * g.n[d];
      nl->N *= g.n[d];
    }
    BKTS_REQUIRE(nl->N < ((int64_t)1 << 31), "grid too large (N >= 2^31)");
    for (int i = 0; i < 4; ++i) {
      g.dc[i] = c->dcoef[i];
      g.rc[i] = c->rcoef[i];
    }
    bkts_fv_coeffs lc{};
    lc.kappa_const = 1.0;
    for (int f = 0; f < 6; ++f) {
      BKTS_REQUIRE(c->bc_type[f] == BKTS_BC_DIRICHLET || c->bc_type[f] == BKTS_BC_NEUMANN, "bad bc_type[%d]", f);
      g.bc_type[f] = c->bc_type[f];
      g.bc_val[f] = c->bc_value[f];
      lc.bc_type[f] = c->bc_type[f];
    }
    nl->jac = fv_assemble(ctx, grid, &lc, BKTS_FMT_SELL);  // the stencil sparsity
  } catch (...) {
    delete nl;
    throw;
  }
  return nl;
}

void nl_eval(bkts_ctx ctx, const bkts_nlop_s& nl, int k, const double* Y, int ldy, double* F, int ldf) {
  const int64_t n = nl.N * k;
  if (n == 0) return;
  ProfScope prof(ctx, BKTS_K_OTHER, 16.0 * n);
  launch(ctx, nl_eval_kernel, dim3((n + 255) / 256), dim3(256), 0, nl.nd, nl.N, k, Y, ldy, F, ldf);
  BKTS_HIP(hipGetLastError());
}

void nl_mass(bkts_ctx ctx, const bkts_nlop_s& nl, int k, const double* Y, int ldy, double* M, int ldm) {
  const int64_t n = nl.N * k;
  if (n == 0) return;
  ProfScope prof(ctx, BKTS_K_OTHER, 16.0 * n);
  launch(ctx, nl_mass_kernel, dim3((n + 255) / 256), dim3(256), 0, nl.nd, nl.N, k, Y, ldy, M, ldm);
  BKTS_HIP(hipGetLastError());
}

bkts_nlop richards_create(bkts_ctx ctx, const bkts_grid* grid, const double* ks, const bkts_richards_params* p) {
  BKTS_REQUIRE(grid && ks && p, "grid, ks and params must not be NULL");
  BKTS_REQUIRE(grid->dim >= 1 && grid->dim <= 3, "grid dim must be 1, 2 or 3");
  BKTS_REQUIRE(p->n > 1.0 && p->alpha > 0.0 && p->theta_s > p->theta_r && p->theta_r >= 0.0,
               "van Genuchten parameters need n > 1, alpha > 0, theta_s > theta_r >= 0");
  BKTS_REQUIRE(p->top == BKTS_RI_DIRICHLET || p->top == BKTS_RI_NO_FLOW, "top must be Dirichlet or no flow");
  BKTS_REQUIRE(p->bottom == BKTS_RI_FREE_DRAINAGE || p->bottom == BKTS_RI_NO_FLOW,
               "bottom must be free drainage or no flow");
  BKTS_REQUIRE(p->lin_L >= 0.0, "lin_L must be >= 0");
  auto* nl = new bkts_nlop_s();
  try {
    nl->ctx = ctx;
    NlDev& g = nl->nd;
    g.kind = 1;
    g.dim = grid->dim;
    nl->N = 1;
    for (int d = 0; d < 3; ++d) {
      g.n[d] = d < grid->dim ? grid->n[d] : 1;
      BKTS_REQUIRE(g.n[d] >= 1, "grid n[%d] must be >= 1", d);
      g.w[d] = (double)g.n[d] * g.n[d];
      nl->N *= g.n[d];
    }
    BKTS_REQUIRE(nl->N < ((int64_t)1 << 31), "grid too large (N >= 2^31)");
    g.tr = p->theta_r;
    g.ts = p->theta_s;
    g.alpha = p->alpha;
    g.vn = p->n;
    g.vm = 1.0 - 1.0 / p->n;
    g.top_dirichlet = p->top == BKTS_RI_DIRICHLET;
    g.bottom_drain = p->bottom == BKTS_RI_FREE_DRAINAGE;
    g.top_g = p->top_value;
    {  // kr(top_value) on the host, by the same closure
      const double se = p->top_value < 0.0 ? std::pow(1.0 + std::pow(-p->alpha * p->top_value, p->n), -g.vm) : 1.0;
      const double s = (g.tr + (g.ts - g.tr) * se) / g.ts;
      const double gg = 1.0 - std::pow(1.0 - std::pow(s, 1.0 / g.vm), g.vm);
      g.top_kr = std::sqrt(s) * gg * gg;
    }
    g.hz = 1.0 / g.n[g.dim - 1];
    g.lin_L = p->lin_L;
    nl->ks.alloc(sizeof(double) * nl->N);
    BKTS_HIP(hipMemcpyAsync(nl->ks.p, ks, sizeof(double) * nl->N, hipMemcpyDeviceToDevice, ctx->stream));
    ctx->sync();  // the caller may release ks on return
    g.ks = nl->ks.as<double>();
    bkts_fv_coeffs lc{};
    lc.kappa_const = 1.0;
    for (int f = 0; f < 6; ++f) lc.bc_type[f] = BKTS_BC_NEUMANN;
    nl->jac = fv_assemble(ctx, grid, &lc, BKTS_FMT_SELL);  // the stencil sparsity
  } catch (...) {
    delete nl;
    throw;
  }
  return nl;
}

void nl_jacobian(bkts_ctx ctx, bkts_nlop_s& nl, const double* u, int ldu, double alpha, double beta) {
  bkts_op J = nl.jac;
  {
    ProfScope prof(ctx, BKTS_K_OTHER, 8.0 * J->nnz + 12.0 * nl.N);
    launch(ctx, nl_jac_kernel, dim3((nl.N + 255) / 256), dim3(256), 0, nl.nd, nl.N, u, ldu, alpha,
                       beta, J->rowptr.as<int32_t>(), J->val.as<double>());
    BKTS_HIP(hipGetLastError());
  }
  op_refresh_values(J);
}

void nl_residual(bkts_ctx ctx, const bkts_nlop_s& nl, int k, const double* Y, int ldy, const double* A1,
                 const double* A2, const double* B0, int ldb0, int nb0, const int* b0_to_col, double* R, int ldr,
                 double* nrm) {
  BKTS_REQUIRE(nb0 >= 0 && nb0 <= 8, "at most 8 B0 columns");
  NlResArgs a{};
  a.g = nl.nd;
  a.N = nl.N;
  a.k = k;
  a.Y = Y;
  a.ldy = ldy;
  a.A1 = A1;
  a.A2 = A2;
  a.B0 = B0;
  a.ldb0 = ldb0;
  a.nb0 = B0 ? nb0 : 0;
  for (int j = 0; j < 8; ++j) a.b0col[j] = j < a.nb0 ? b0_to_col[j] : -1;
  a.R = R;
  a.ldr = ldr;
  if (nl.nd.kind == 1) {  // Richards: theta and kr once per entry, then the flux pass reads them
    double* th = ctx->ws.get<double>("ri_theta", (size_t)nl.N * k);
    double* kr = ctx->ws.get<double>("ri_kr", (size_t)nl.N * k);
    const int64_t n = nl.N * k;
    ProfScope prof(ctx, BKTS_K_OTHER, 24.0 * n);
    launch(ctx, ri_cache_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, nl.nd, nl.N, k, Y, ldy, th, kr);
    BKTS_HIP(hipGetLastError());
    a.th = th;
    a.kr = kr;
  }
  switch (k <= 1 ? 1 : k <= 2 ? 2 : k <= 4 ? 4 : k <= 8 ? 8 : k <= 16 ? 16 : 32) {
    case 1: launch_nlres<1>(ctx, a, nrm); break;
    case 2: launch_nlres<2>(ctx, a, nrm); break;
    case 4: launch_nlres<4>(ctx, a, nrm); break;
    case 8: launch_nlres<8>(ctx, a, nrm); break;
    case 16: launch_nlres<16>(ctx, a, nrm); break;
    default: launch_nlres<32>(ctx, a, nrm); break;
  }
}

}  // namespace bkts

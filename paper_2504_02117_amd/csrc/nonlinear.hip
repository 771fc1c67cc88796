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

// ---- van Genuchten closure (eq. RelationshipsThetaK), s = theta / theta_s as printed.
// With a = -alpha psi (psi < 0), t = a^n, S_e = (1 + t)^(-m), m = 1 - 1/n, w = 1 - s^(1/m), g = 1 - w^m:
//   theta = theta_r + (theta_s - theta_r) S_e,        kr = s^(1/2) g^2,
//   dS_e/dpsi = alpha m n a^(n-1) (1 + t)^(-m-1) = alpha m n (t / a) S_e / (1 + t),
//   dkr/dpsi = (s^(-1/2) g^2 / 2 + 2 s^(1/2) g w^(m-1) s^(1/m-1)) ds/dpsi,  w^(m-1) s^(1/m-1) = (w^m / w)(s^(1/m) / s).
// Every power goes through one logarithm and one exponential, and the derivatives reuse the powers
// of the values. For n = 2 (m = 1/2, 1/m = 2) the powers are products and square roots.
struct VgVals {
  double theta, kr, dtheta, dkr;
};

__device__ __forceinline__ double vg_se_t(const NlDev& g, double a, double& t) {
  if (g.vn == 2.0) {
    t = a * a;
    return 1.0 / sqrt(1.0 + t);
  }
  t = exp(g.vn * log(a));
  return exp(-g.vm * log1p(t));
}

template <bool DERIV>
__device__ __forceinline__ VgVals vg_eval(const NlDev& g, double psi) {
  VgVals v;
  if (!(psi < 0.0)) {  // saturated: S_e = 1, s = 1, w = 0
    v.theta = g.ts;
    v.kr = 1.0;
    v.dtheta = 0.0;
    v.dkr = 0.0;
    return v;
  }
  const double a = -g.alpha * psi;
  double t;
  const double se = vg_se_t(g, a, t);
  v.theta = g.tr + (g.ts - g.tr) * se;
  const double s = v.theta / g.ts;
  const bool two = g.vn == 2.0;
  const double s1m = two ? s * s : exp(log(s) / g.vm);  // s^(1/m)
  const double w = 1.0 - s1m;
  const double wm = w > 0.0 ? (two ? sqrt(w) : exp(g.vm * log(w))) : 0.0;  // w^m
  const double gg = 1.0 - wm, rs = sqrt(s);
  v.kr = rs * gg * gg;
  v.dtheta = 0.0;
  v.dkr = 0.0;
  if (DERIV) {
    const double an1 = two ? a : (a > 0.0 ? t / a : 0.0);  // a^(n-1)
    v.dtheta = (g.ts - g.tr) * g.alpha * g.vm * g.vn * an1 * se / (1.0 + t);
    const double ds = v.dtheta / g.ts;
    const double dg = w > 0.0 ? (wm / w) * (s1m / s) : 0.0;
    v.dkr = (0.5 / rs * gg * gg + rs * 2.0 * gg * dg) * ds;
  }
  return v;
}

__device__ __forceinline__ double vg_theta(const NlDev& g, double psi) {
  if (!(psi < 0.0)) return g.ts;
  double t;
  return g.tr + (g.ts - g.tr) * vg_se_t(g, -g.alpha * psi, t);
}
__device__ __forceinline__ double vg_kr(const NlDev& g, double psi) { return vg_eval<false>(g, psi).kr; }
__device__ __forceinline__ double mass_at(const NlDev& g, double u) { return g.kind == 1 ? vg_theta(g, u) : u; }

__device__ __forceinline__ double harm(double a, double b) { return a + b > 0.0 ? 2.0 * a * b / (a + b) : 0.0; }

// The six face neighbours of cell r: their rows (the cell itself for a face on the border or beyond
// the grid's dimension) and whether the face is interior.
struct Faces {
  int i[3];
  int64_t q[6];
  bool in[6];
};

__device__ __forceinline__ Faces faces_of(const NlDev& g, int64_t r) {
  Faces F;
  coords(g, r, F.i);
  int64_t st = 1;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    F.in[2 * d] = d < g.dim && F.i[d] > 0;
    F.in[2 * d + 1] = d < g.dim && F.i[d] < g.n[d] - 1;
    F.q[2 * d] = F.in[2 * d] ? r - st : r;
    F.q[2 * d + 1] = F.in[2 * d + 1] ? r + st : r;
    st *= g.n[d];
  }
  return F;
}

// Richards f(psi)_r for the column of u with stride ld, kr of cell q from kr_at(q). Every neighbour
// value is loaded before any is used (border faces load the cell itself and add nothing), so the
// loads of one cell are in flight together; faces are summed in axis order, low side first.
// The transmissibility harm(Ks_P, Ks_Q) / h_d^2 of every face of cell r (the low face along d is the
// high face of the neighbour below), and Ks_r.
__device__ __forceinline__ double face_t(const NlDev& g, int64_t r, const Faces& F, double (&T)[6]) {
  const double2 a = *reinterpret_cast<const double2*>(g.tf + 4 * r);
  const double2 b = *reinterpret_cast<const double2*>(g.tf + 4 * r + 2);
  T[1] = a.x;
  T[3] = a.y;
  T[5] = b.x;
#pragma unroll
  for (int d = 0; d < 3; ++d) T[2 * d] = g.tf[4 * F.q[2 * d] + d];
  return b.y;
}

template <class KrAt>
__device__ __forceinline__ double ri_flux(const NlDev& g, const double* u, int ld, int64_t r, KrAt kr_at) {
  const Faces F = faces_of(g, r);
  const double up = u[r * ld], krp = kr_at(r);
  double uq[6], kq[6], T[6];
#pragma unroll
  for (int e = 0; e < 6; ++e) {
    uq[e] = u[F.q[e] * ld];
    kq[e] = kr_at(F.q[e]);
  }
  const double ksp = face_t(g, r, F, T);
  const int zd = g.dim - 1;
  const double zp = (F.i[zd] + 0.5) * g.hz, Hp = up + zp;
  double f = 0.0;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
#pragma unroll
    for (int side = 0; side < 2; ++side) {
      const int e = 2 * d + side;
      if (F.in[e]) {
        const double Hq = uq[e] + (d == zd ? zp + (side == 0 ? -g.hz : g.hz) : zp);
        f += T[e] * 0.5 * (krp + kq[e]) * (Hp - Hq);
      } else if (d == zd && side == 1 && g.top_dirichlet) {
        f += 2.0 * ksp * 0.5 * (krp + g.top_kr) * (Hp - (g.top_g + 1.0)) * g.w[d];
      } else if (d == zd && side == 0 && g.bottom_drain) {
        f += ksp * krp / g.hz;
      }
    }
  }
  return f;
}

// Diffusion-reaction f(u)_r for the column of u with stride ld, loads first as in ri_flux.
__device__ __forceinline__ double dr_flux(const NlDev& g, const double* u, int ld, int64_t r) {
  const Faces F = faces_of(g, r);
  const double up = u[r * ld];
  double uq[6];
#pragma unroll
  for (int e = 0; e < 6; ++e) uq[e] = u[F.q[e] * ld];
  const double Dp = poly(g.dc, up);
  double f = -poly(g.rc, up);
#pragma unroll
  for (int d = 0; d < 3; ++d) {
#pragma unroll
    for (int side = 0; side < 2; ++side) {
      const int e = 2 * d + side;
      if (F.in[e]) {
        f += 0.5 * (Dp + poly(g.dc, uq[e])) * (up - uq[e]) * g.w[d];
      } else if (d < g.dim && g.bc_type[e] == BKTS_BC_DIRICHLET) {
        const double gv = g.bc_val[e];
        f += 0.5 * (Dp + poly(g.dc, gv)) * (up - gv) * 2.0 * g.w[d];
      }
    }
  }
  return f;
}

// theta and kr of every entry of the first k columns of Y, into TH and KR (N x k, contiguous)
__global__ void ri_cache_kernel(NlDev g, int64_t N, int k, const double* Y, int ldy, double* TH, double* KR) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N * k) return;
  const int64_t r = i / k;
  const int c = (int)(i - r * k);
  const VgVals v = vg_eval<false>(g, Y[r * ldy + c]);
  TH[i] = v.theta;
  KR[i] = v.kr;
}

// Per cell r: harm(Ks_r, Ks_q) / h_d^2 for the next cell q along x, y, z (0 where there is none), Ks_r.
__global__ void ri_faces_kernel(NlDev g, int64_t N, const double* ks, double* tf) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= N) return;
  const Faces F = faces_of(g, r);
  const double kp = ks[r];
#pragma unroll
  for (int d = 0; d < 3; ++d) tf[4 * r + d] = F.in[2 * d + 1] ? harm(kp, ks[F.q[2 * d + 1]]) * g.w[d] : 0.0;
  tf[4 * r + 3] = kp;
}

// f(u)_r for the column of u with stride ld (u[q * ld])
__device__ double f_at(const NlDev& g, const double* u, int ld, int64_t r) {
  if (g.kind == 1) return ri_flux(g, u, ld, r, [&](int64_t q) { return vg_kr(g, u[q * ld]); });
  return dr_flux(g, u, ld, r);
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

// Row r of the Richards Jacobian alpha m'(u) + beta Df(u) (m' = theta' or lin_L): the diagonal and
// the off-diagonal entry of every face (interior faces only carry one).
__device__ __forceinline__ void ri_jac_row(const NlDev& g, const double* u, int ldu, int64_t r, const Faces& F,
                                           double alpha, double beta, double& diag, double (&off)[6]) {
  const double up = u[r * ldu];
  double uq[6], T[6];
#pragma unroll
  for (int e = 0; e < 6; ++e) uq[e] = u[F.q[e] * ldu];
  const double ksp = face_t(g, r, F, T);
  const VgVals vp = vg_eval<true>(g, up);
  const double krp = vp.kr, dkrp = vp.dkr;
  const int zd = g.dim - 1;
  const double zp = (F.i[zd] + 0.5) * g.hz, Hp = up + zp;
  double dd = 0.0;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
#pragma unroll
    for (int side = 0; side < 2; ++side) {
      const int e = 2 * d + side;
      off[e] = 0.0;
      if (F.in[e]) {
        const VgVals vq = vg_eval<true>(g, uq[e]);
        const double Hq = uq[e] + (d == zd ? zp + (side == 0 ? -g.hz : g.hz) : zp);
        const double wk = T[e];
        const double m = 0.5 * (krp + vq.kr), dH = Hp - Hq;
        dd += wk * (m + 0.5 * dkrp * dH);
        off[e] = beta * wk * (-m + 0.5 * vq.dkr * dH);
      } else if (d == zd && side == 1 && g.top_dirichlet) {
        dd += 2.0 * ksp * (0.5 * (krp + g.top_kr) + 0.5 * dkrp * (Hp - (g.top_g + 1.0))) * g.w[d];
      } else if (d == zd && side == 0 && g.bottom_drain) {
        dd += ksp * dkrp / g.hz;
      }
    }
  }
  const double mp = g.lin_L > 0.0 ? g.lin_L : vp.dtheta;
  diag = alpha * mp + beta * dd;
}

// Row r of the diffusion-reaction Jacobian alpha I + beta Df(u).
__device__ __forceinline__ void dr_jac_row(const NlDev& g, const double* u, int ldu, int64_t r, const Faces& F,
                                           double alpha, double beta, double& diag, double (&off)[6]) {
  const double up = u[r * ldu];
  double uq[6];
#pragma unroll
  for (int e = 0; e < 6; ++e) uq[e] = u[F.q[e] * ldu];
  const double Dp = poly(g.dc, up), dDp = dpoly(g.dc, up);
  double dd = -dpoly(g.rc, up);
#pragma unroll
  for (int d = 0; d < 3; ++d) {
#pragma unroll
    for (int side = 0; side < 2; ++side) {
      const int e = 2 * d + side;
      off[e] = 0.0;
      if (F.in[e]) {
        const double Dq = poly(g.dc, uq[e]), dDq = dpoly(g.dc, uq[e]);
        const double Df = 0.5 * (Dp + Dq), diff = up - uq[e];
        dd += (Df + 0.5 * dDp * diff) * g.w[d];
        off[e] = beta * ((-Df + 0.5 * dDq * diff) * g.w[d]);
      } else if (d < g.dim && g.bc_type[e] == BKTS_BC_DIRICHLET) {
        const double gv = g.bc_val[e];
        dd += (0.5 * (Dp + poly(g.dc, gv)) + 0.5 * dDp * (up - gv)) * 2.0 * g.w[d];
      }
    }
  }
  diag = alpha + beta * dd;
}

// Row r of J = alpha m'(u) + beta Df(u), written in the stencil's sorted column order
// (z-, y-, x-, diagonal, x+, y+, z+) starting at val[rowptr[r]].
__global__ void nl_jac_kernel(NlDev g, int64_t N, const double* u, int ldu, double alpha, double beta,
                              const int32_t* rowptr, double* val) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= N) return;
  const Faces F = faces_of(g, r);
  double diag, off[6];
  if (g.kind == 1)
    ri_jac_row(g, u, ldu, r, F, alpha, beta, diag, off);
  else
    dr_jac_row(g, u, ldu, r, F, alpha, beta, diag, off);
  int64_t p = rowptr[r];
  for (int d = g.dim - 1; d >= 0; --d)
    if (F.in[2 * d]) val[p++] = off[2 * d];
  val[p++] = diag;
  for (int d = 0; d < g.dim; ++d)
    if (F.in[2 * d + 1]) val[p++] = off[2 * d + 1];
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

// Tiles of the window residual: 256 / KP rows, one per thread and column; m(Y) and F(Y) of the tile
// staged in LDS for the right-multiplications by A1^T and A2^T, whose transposes sit in LDS too.
template <int KP>
struct NlResGeom {
  static constexpr int RT = 256 / KP;
  static constexpr int LDL = TileGeom<KP>::LDL;
  static constexpr int TILE = 2 * RT * LDL;
  static constexpr int LDS = TILE + 2 * KP * KP;
};

// KIND 0: diffusion-reaction (m = identity); KIND 1: Richards (theta and kr read from the cache).
template <int KP, int KIND>
__global__ __launch_bounds__(256) void nl_residual_kernel(NlResArgs a) {
  using G = NlResGeom<KP>;
  static_assert(G::TILE >= 4 * KP, "the block reduction reuses the tile");
  __shared__ __align__(16) double lds[G::LDS];
  double* Ml = lds;
  double* Fl = lds + G::RT * G::LDL;
  double* At1 = lds + G::TILE;  // At1[j * KP + c] = A1[c][j]
  double* At2 = At1 + KP * KP;
  const int t = threadIdx.x, c = t % KP, row = t / KP;
  for (int e = t; e < KP * KP; e += 256) {
    const int j = e / KP, cc = e % KP;
    const bool in = cc < a.k && j < a.k;
    At1[e] = in ? a.A1[cc * a.k + j] : 0.0;
    At2[e] = in ? a.A2[cc * a.k + j] : 0.0;
  }
  const int64_t slot = dev::xcd_slot(blockIdx.x, gridDim.x);
  const int64_t ntiles = (a.N + G::RT - 1) / G::RT;
  const bool cok = c < a.k;
  const int cc = cok ? c : 0;  // padding columns read column 0 and discard it
  int b0j = -1;
  for (int j = 0; j < a.nb0; ++j)
    if (a.b0col[j] == c) b0j = j;
  double nacc[1] = {0.0};
  const int64_t tend = (slot + 1) * a.tps < ntiles ? (slot + 1) * a.tps : ntiles;
  for (int64_t tile = slot * a.tps; tile < tend; ++tile) {
    const int64_t gr = tile * G::RT + row;
    const bool ok = gr < a.N && cok;
    const int64_t rr = gr < a.N ? gr : 0;  // rows past the end evaluate row 0 and discard it
    double mv, fv;
    if constexpr (KIND == 1) {
      const double* kr = a.kr + cc;
      mv = a.th[rr * a.k + cc];
      fv = ri_flux(a.g, a.Y + cc, a.ldy, rr, [&](int64_t q) { return kr[q * a.k]; });
    } else {
      mv = a.Y[rr * a.ldy + cc];
      fv = dr_flux(a.g, a.Y + cc, a.ldy, rr);
    }
    Ml[row * G::LDL + c] = ok ? mv : 0.0;
    Fl[row * G::LDL + c] = ok ? fv : 0.0;
    __syncthreads();
    if (ok) {
      const double* pm = Ml + row * G::LDL;
      const double* pf = Fl + row * G::LDL;
      double s1 = 0.0, s2 = 0.0;
#pragma unroll 4
      for (int j = 0; j < KP; ++j) s1 = fma(pm[j], At1[j * KP + c], s1);
#pragma unroll 4
      for (int j = 0; j < KP; ++j) s2 = fma(pf[j], At2[j * KP + c], s2);
      double r = s1 + s2;
      if (b0j >= 0) r -= a.B0[gr * a.ldb0 + b0j];
      a.R[gr * a.ldr + c] = r;
      nacc[0] = fma(r, r, nacc[0]);
    }
    __syncthreads();
  }
  dev::block_reduce_store<KP, 1>(nacc, lds, a.partials, gridDim.x, slot);
}

template <int KP>
void launch_nlres(bkts_ctx ctx, NlResArgs a, double* nrm) {
  using G = NlResGeom<KP>;
  const int64_t ntiles = (a.N + G::RT - 1) / G::RT;
  const int64_t cap = 8 * (int64_t)ctx->num_cu;  // latency-bound gathers: many workgroups in flight
  int64_t ns = ntiles < cap ? ntiles : cap;
  if (ns < 1) ns = 1;
  a.tps = (ntiles + ns - 1) / ns;
  a.partials = ctx->ws.get<double>("nlres_partials", (size_t)KP * ns);
  ProfScope prof(ctx, BKTS_K_RESIDUAL, 16.0 * a.N * a.k + 8.0 * a.N * a.nb0);
  if (a.g.kind == 1)
    launch(ctx, (nl_residual_kernel<KP, 1>), dim3(ns), dim3(256), 0, a);
  else
    launch(ctx, (nl_residual_kernel<KP, 0>), dim3(ns), dim3(256), 0, a);
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
    nl->jac->mg_sym = sym_stencil_create(*nl->jac);          // for BKTS_PREC_MG
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
    g.ks = nl->ks.as<double>();
    nl->tf.alloc(sizeof(double) * 4 * nl->N);
    g.tf = nl->tf.as<double>();
    launch(ctx, ri_faces_kernel, dim3((unsigned)((nl->N + 255) / 256)), dim3(256), 0, g, nl->N, g.ks, nl->tf.as<double>());
    BKTS_HIP(hipGetLastError());
    ctx->sync();  // the caller may release ks on return, and other streams may use the operator
    bkts_fv_coeffs lc{};
    lc.kappa_const = 1.0;
    for (int f = 0; f < 6; ++f) lc.bc_type[f] = BKTS_BC_NEUMANN;
    nl->jac = fv_assemble(ctx, grid, &lc, BKTS_FMT_SELL);  // the stencil sparsity
    nl->jac->mg_sym = sym_stencil_create(*nl->jac);          // for BKTS_PREC_MG
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
  J->mg_sym_stale = true;
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

// Geometric multigrid V-cycle for A = a I + b K on structured grids, as the preconditioner of block
// CG (the paper solves its inner systems with AMG-preconditioned Krylov methods, Sec. 4.1; this is
// a geometric counterpart built from the index-free stencil form of K).
//
// Hierarchy: level 0 is the fine grid; level l+1 aggregates 2 x 2 x 2 cells of level l (one cell
// along an axis of odd length at its end).  With P the piecewise-constant prolongation, every level
// holds the Galerkin products K_{l+1} = P^T K_l P and M_{l+1} = P^T M_l P (M_0 = I), which keep the
// 7-point form: a coarse diagonal collects its children's diagonals plus twice the couplings inside
// the aggregate, a coarse coupling sums the fine couplings across the aggregate face, and the coarse
// mass counts the fine cells.  A_l = a M_l + b K_l is formed on the fly, so one hierarchy serves
// every (a, b).
//
// V-cycle (symmetric, so it preconditions CG): on level l with right-hand side f,
//   x = w D^-1 f                     (one damped Jacobi sweep from zero)
//   f_{l+1} = P^T (f - A x)          (residual and restriction, one pass)
//   x_{l+1} = V-cycle(l + 1, f_{l+1})
//   z = x + P x_{l+1};  z += w D^-1 (f - A z)   (prolongation and post-sweep, one pass)
// with the pre-smoothed x recomputed wherever it is needed instead of stored, and on the coarsest
// level (at most 64 cells) a fixed number of damped Jacobi sweeps in one workgroup.
#include <memory>
#include <vector>

#include "devcommon.hpp"
#include "internal.hpp"

namespace bkts {

struct MgLevel {
  int n[3];
  int64_t N;
  DevBuf c64, c32;  // 5 arrays of N: dK, m, o_x, o_y, o_z  (o_d[r] = K[r, r + s_d], 0 past the + face)
  DevBuf di64, di32;  // 1 / (a m + b dK) for the (a, b) of the last V-cycle
};

struct MgHier {
  std::vector<MgLevel> lv;
  double a = 0.0, b = 0.0;  // the pair the inverse diagonals hold (0, 0: none yet)
};

namespace {

constexpr int kCoarsestMax = 64;  // cells of the coarsest level
constexpr int kCoarseSweeps = 12;
constexpr double kOmega = 0.8;

struct Geo {
  int nx, ny, nz;
  int64_t N;
  int64_t sx, sy, sz;  // 1, nx, nx*ny
};

Geo geo_of(const MgLevel& l) {
  Geo g{l.n[0], l.n[1], l.n[2], l.N, 1, l.n[0], (int64_t)l.n[0] * l.n[1]};
  return g;
}

__device__ __forceinline__ void coords(const Geo& g, int64_t r, int& ix, int& iy, int& iz) {
  const uint32_t q = (uint32_t)r / (uint32_t)g.nx;
  ix = (int)((uint32_t)r - q * (uint32_t)g.nx);
  const uint32_t q2 = q / (uint32_t)g.ny;
  iy = (int)(q - q2 * (uint32_t)g.ny);
  iz = (int)q2;
}

// Level-0 arrays from the operator's stencil form: axis d takes the stencil array whose offset is
// s_d when the axis has two or more cells, zeros otherwise; the mass is one per cell.
__global__ void mg_level0(int64_t N, int na, const double* st, int sel0, int sel1, int sel2, double* c) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= N) return;
  c[r] = st[r];
  c[N + r] = 1.0;
  const int sel[3] = {sel0, sel1, sel2};
  for (int d = 0; d < 3; ++d) c[(2 + d) * N + r] = sel[d] >= 0 ? st[(1 + sel[d]) * N + r] : 0.0;
  (void)na;
}

// Galerkin coarsening of (dK, m, o) from level f to level c, one thread per coarse cell.
__global__ void mg_coarsen(Geo f, Geo c, const double* cf, double* cc) {
  const int64_t R = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (R >= c.N) return;
  int X, Y, Z;
  coords(c, R, X, Y, Z);
  double dk = 0.0, m = 0.0, o[3] = {0.0, 0.0, 0.0};
  const int64_t Nf = f.N;
  for (int dz = 0; dz < 2; ++dz) {
    const int iz = 2 * Z + dz;
    if (iz >= f.nz) continue;
    for (int dy = 0; dy < 2; ++dy) {
      const int iy = 2 * Y + dy;
      if (iy >= f.ny) continue;
      for (int dx = 0; dx < 2; ++dx) {
        const int ix = 2 * X + dx;
        if (ix >= f.nx) continue;
        const int64_t i = ix + f.sy * iy + f.sz * iz;
        dk += cf[i];
        m += cf[Nf + i];
        const int own[3] = {dx, dy, dz};
        const int pos[3] = {ix, iy, iz};
        const int len[3] = {f.nx, f.ny, f.nz};
        for (int d = 0; d < 3; ++d) {
          const double od = cf[(2 + d) * Nf + i];  // coupling to the + neighbour along d
          if (pos[d] + 1 >= len[d]) continue;      // no neighbour (od is zero)
          if (own[d] == 0)
            dk += 2.0 * od;  // the neighbour is the other child of this aggregate
          else
            o[d] += od;      // the neighbour belongs to the next aggregate along d
        }
      }
    }
  }
  cc[R] = dk;
  cc[c.N + R] = m;
  for (int d = 0; d < 3; ++d) cc[(2 + d) * c.N + R] = o[d];
}

// di = 1 / (a m + b dK) on one level, FP64 and FP32.
__global__ void mg_dinv(int64_t N, const double* c, double a, double b, double* d64, float* d32) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= N) return;
  const double v = 1.0 / (a * c[N + r] + b * c[r]);
  d64[r] = v;
  d32[r] = (float)v;
}

__global__ void mg_to_f32(int64_t n, const double* in, float* out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = (float)in[i];
}

template <typename T>
struct LvArgs {
  Geo g;
  const T* c;   // 5 arrays of N
  const T* di;  // inverse diagonal of A on this level
  T a, b, w;
  int k;
};

// Damped Jacobi from zero: x[r] = w f[r] / dA[r], for the CW columns starting at c0.
template <typename T, int CW>
__device__ __forceinline__ void pre_x(const LvArgs<T>& L, const T* f, int64_t r, int c0, T (&x)[CW]) {
  const T s = L.w * L.di[r];
#pragma unroll
  for (int j = 0; j < CW; ++j) x[j] = s * f[r * L.k + c0 + j];
}

// (A y)[r] for the CW columns at c0, where y at any cell q is produced by ycell(q, out[CW]).
template <typename T, int CW, typename Y>
__device__ __forceinline__ void apply_row(const LvArgs<T>& L, int64_t r, int ix, int iy, int iz, const T (&yr)[CW],
                                          Y ycell, T (&out)[CW]) {
  const Geo& g = L.g;
  const int64_t N = g.N;
  const T dA = T(1) / L.di[r];  // the diagonal from its cached inverse: no dK or mass read
#pragma unroll
  for (int j = 0; j < CW; ++j) out[j] = dA * yr[j];
  const int pos[3] = {ix, iy, iz};
  const int len[3] = {g.nx, g.ny, g.nz};
  const int64_t st[3] = {g.sx, g.sy, g.sz};
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const T* od = L.c + (2 + d) * N;
    if (pos[d] + 1 < len[d]) {
      const T cu = L.b * od[r];
      T y[CW];
      ycell(r + st[d], y);
#pragma unroll
      for (int j = 0; j < CW; ++j) out[j] = fma(cu, y[j], out[j]);
    }
    if (pos[d] > 0) {
      const T cl = L.b * od[r - st[d]];
      T y[CW];
      ycell(r - st[d], y);
#pragma unroll
      for (int j = 0; j < CW; ++j) out[j] = fma(cl, y[j], out[j]);
    }
  }
}

// fc = P^T (f - A x) with x = w D^-1 f.  A workgroup covers a strip of 32 coarse cells along x: its
// 256 threads are the 64 x 2 x 2 fine cells of those aggregates (consecutive threads on consecutive
// cells of one grid line), each forms its own residual, and the 8 residuals of an aggregate are
// summed through LDS in a fixed order.  Grid: (ceil(ncx / 32), ncy, ncz).
template <typename T, int CW>
__global__ __launch_bounds__(256) void mg_restrict_kernel(LvArgs<T> L, Geo c, const T* __restrict__ f,
                                                          T* __restrict__ fc) {
  __shared__ T red[CW][256];
  const int t = threadIdx.x;
  const int x = t & 63, y = (t >> 6) & 1, z = t >> 7;
  const int X0 = blockIdx.x * 32, Y = blockIdx.y, Z = blockIdx.z;
  const Geo& g = L.g;
  const int ix = 2 * X0 + x, iy = 2 * Y + y, iz = 2 * Z + z;
  const bool in = ix < g.nx && iy < g.ny && iz < g.nz;
  const int64_t i = in ? ix + g.sy * iy + g.sz * iz : 0;
  for (int c0 = 0; c0 < L.k; c0 += CW) {
    T v[CW];
#pragma unroll
    for (int j = 0; j < CW; ++j) v[j] = T(0);
    if (in) {
      T xi[CW], ax[CW];
      pre_x<T, CW>(L, f, i, c0, xi);
      apply_row<T, CW>(L, i, ix, iy, iz, xi, [&](int64_t q, T(&yq)[CW]) { pre_x<T, CW>(L, f, q, c0, yq); }, ax);
#pragma unroll
      for (int j = 0; j < CW; ++j) v[j] = f[i * L.k + c0 + j] - ax[j];
    }
#pragma unroll
    for (int j = 0; j < CW; ++j) red[j][t] = v[j];
    __syncthreads();
    if (t < 32 && X0 + t < c.nx) {
      const int64_t R = (X0 + t) + c.sy * Y + c.sz * Z;
#pragma unroll
      for (int j = 0; j < CW; ++j) {
        T sum = T(0);
#pragma unroll
        for (int q = 0; q < 8; ++q) sum += red[j][(2 * t + (q & 1)) + 64 * ((q >> 1) & 1) + 128 * (q >> 2)];
        fc[R * L.k + c0 + j] = sum;
      }
    }
    __syncthreads();
  }
}

// z = y + w D^-1 (f - A y) with y = w D^-1 f + P xc, one thread per fine cell.
template <typename T, int CW>
__global__ __launch_bounds__(256) void mg_prolong_kernel(LvArgs<T> L, Geo c, const T* __restrict__ f,
                                                         const T* __restrict__ xc, T* __restrict__ z) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= L.g.N) return;
  int ix, iy, iz;
  coords(L.g, r, ix, iy, iz);
  auto ycell = [&](int64_t q, int qx, int qy, int qz, int c0, T(&y)[CW]) {
    pre_x<T, CW>(L, f, q, c0, y);
    const int64_t P = (qx >> 1) + c.sy * (qy >> 1) + c.sz * (qz >> 1);
#pragma unroll
    for (int j = 0; j < CW; ++j) y[j] += xc[P * L.k + c0 + j];
  };
  for (int c0 = 0; c0 < L.k; c0 += CW) {
    T yr[CW], ay[CW];
    ycell(r, ix, iy, iz, c0, yr);
    apply_row<T, CW>(L, r, ix, iy, iz, yr,
                     [&](int64_t q, T(&y)[CW]) {
                       int qx, qy, qz;
                       coords(L.g, q, qx, qy, qz);
                       ycell(q, qx, qy, qz, c0, y);
                     },
                     ay);
    const T s = L.w * L.di[r];
#pragma unroll
    for (int j = 0; j < CW; ++j) z[r * L.k + c0 + j] = yr[j] + s * (f[r * L.k + c0 + j] - ay[j]);
  }
}

// Coarsest level: kCoarseSweeps damped Jacobi sweeps from zero in one workgroup (x in LDS).
template <typename T>
__global__ __launch_bounds__(256) void mg_coarse_kernel(LvArgs<T> L, const T* __restrict__ f, T* __restrict__ z) {
  __shared__ T xs[2][kCoarsestMax * BKTS_MAX_K];
  const int64_t n = L.g.N * L.k;
  for (int64_t e = threadIdx.x; e < n; e += blockDim.x) {
    const int64_t r = e / L.k;
    xs[0][e] = L.w * f[e] * L.di[r];
  }
  __syncthreads();
  int cur = 0;
  for (int it = 1; it < kCoarseSweeps; ++it) {
    for (int64_t e = threadIdx.x; e < n; e += blockDim.x) {
      const int64_t r = e / L.k;
      const int col = (int)(e - r * L.k);
      int ix, iy, iz;
      coords(L.g, r, ix, iy, iz);
      T yr[1] = {xs[cur][e]}, ay[1];
      apply_row<T, 1>(L, r, ix, iy, iz, yr, [&](int64_t q, T(&y)[1]) { y[0] = xs[cur][q * L.k + col]; }, ay);
      xs[cur ^ 1][e] = yr[0] + L.w * (f[e] - ay[0]) * L.di[r];
    }
    __syncthreads();
    cur ^= 1;
  }
  for (int64_t e = threadIdx.x; e < n; e += blockDim.x) z[e] = xs[cur][e];
}

int chunk_width(int k) { return k % 4 == 0 ? 4 : (k % 2 == 0 ? 2 : 1); }

template <typename T>
LvArgs<T> lv_args(const MgLevel& l, int k, double a, double b) {
  LvArgs<T> L;
  L.g = geo_of(l);
  if constexpr (sizeof(T) == 8) {
    L.c = l.c64.as<double>();
    L.di = l.di64.as<double>();
  } else {
    L.c = l.c32.as<float>();
    L.di = l.di32.as<float>();
  }
  L.a = (T)a;
  L.b = (T)b;
  L.w = (T)kOmega;
  L.k = k;
  return L;
}

template <typename T>
void vcycle(bkts_ctx ctx, const MgHier& h, int lvl, int k, double a, double b, const T* f, T* z) {
  const MgLevel& l = h.lv[lvl];
  const LvArgs<T> L = lv_args<T>(l, k, a, b);
  const double sv = sizeof(T);
  if (lvl + 1 == (int)h.lv.size()) {
    ProfScope prof(ctx, BKTS_K_MG_COARSE, sv * (2.0 * l.N * k + 4.0 * l.N));
    launch(ctx, (mg_coarse_kernel<T>), dim3(1), dim3(256), 0, L, f, z);
    return;
  }
  const MgLevel& lc = h.lv[lvl + 1];
  const Geo gc = geo_of(lc);
  const std::string tag = std::to_string(lvl + 1) + (sizeof(T) == 8 ? "d" : "s");
  T* fc = ctx->ws.get<T>("mg_f" + tag, (size_t)lc.N * k);
  T* xc = ctx->ws.get<T>("mg_x" + tag, (size_t)lc.N * k);
  const int cw = chunk_width(k);
  const dim3 gr((unsigned)((lc.n[0] + 31) / 32), (unsigned)lc.n[1], (unsigned)lc.n[2]);
  const dim3 gp((unsigned)((l.N + 255) / 256));
  {  // algorithmic bytes: f, the inverse diagonal and the 3 coupling arrays read, the coarse f written
    ProfScope prof(ctx, lvl == 0 ? BKTS_K_MG_RESTRICT : BKTS_K_MG_COARSE,
                   sv * (1.0 * l.N * k + 4.0 * l.N + 1.0 * lc.N * k));
    if (cw == 4)
      launch(ctx, (mg_restrict_kernel<T, 4>), gr, dim3(256), 0, L, gc, f, fc);
    else if (cw == 2)
      launch(ctx, (mg_restrict_kernel<T, 2>), gr, dim3(256), 0, L, gc, f, fc);
    else
      launch(ctx, (mg_restrict_kernel<T, 1>), gr, dim3(256), 0, L, gc, f, fc);
  }
  vcycle<T>(ctx, h, lvl + 1, k, a, b, fc, xc);
  // algorithmic bytes: f, the coarse x, the inverse diagonal and the 3 coupling arrays read, z written
  ProfScope prof(ctx, lvl == 0 ? BKTS_K_MG_PROLONG : BKTS_K_MG_COARSE,
                 sv * (2.0 * l.N * k + 4.0 * l.N + 1.0 * lc.N * k));
  if (cw == 4)
    launch(ctx, (mg_prolong_kernel<T, 4>), gp, dim3(256), 0, L, gc, f, (const T*)xc, z);
  else if (cw == 2)
    launch(ctx, (mg_prolong_kernel<T, 2>), gp, dim3(256), 0, L, gc, f, (const T*)xc, z);
  else
    launch(ctx, (mg_prolong_kernel<T, 1>), gp, dim3(256), 0, L, gc, f, (const T*)xc, z);
}

}  // namespace

void mg_hier_delete(MgHier* h) { delete h; }

static MgHier* mg_build(bkts_op op) {
  bkts_ctx ctx = op->ctx;
  BKTS_REQUIRE(op->st_na > 0 && op->grid.dim >= 1, "multigrid needs the stencil form (BKTS_FMT_STENCIL)");
  BKTS_REQUIRE(op->N < ((int64_t)1 << 31), "multigrid: grid too large");
  std::unique_ptr<MgHier> h(new MgHier());
  MgLevel l0;
  for (int d = 0; d < 3; ++d) l0.n[d] = d < op->grid.dim ? op->grid.n[d] : 1;
  l0.N = op->N;
  int sel[3] = {-1, -1, -1};
  int64_t s = 1;
  for (int d = 0; d < 3; ++d) {
    if (l0.n[d] >= 2)
      for (int q = 0; q < op->st_na; ++q)
        if (op->st_off[q] == s) sel[d] = q;
    s *= l0.n[d];
  }
  l0.c64.alloc(sizeof(double) * 5 * l0.N);
  l0.c32.alloc(sizeof(float) * 5 * l0.N);
  launch(ctx, mg_level0, dim3((unsigned)((l0.N + 255) / 256)), dim3(256), 0, l0.N, op->st_na,
         op->st_coef.as<double>(), sel[0], sel[1], sel[2], l0.c64.as<double>());
  h->lv.push_back(std::move(l0));
  while (h->lv.back().N > kCoarsestMax && h->lv.size() < 16) {
    const MgLevel& f = h->lv.back();
    MgLevel c;
    for (int d = 0; d < 3; ++d) c.n[d] = (f.n[d] + 1) / 2;
    BKTS_REQUIRE(c.n[1] <= 65535 && c.n[2] <= 65535, "multigrid: grid too tall for the restriction launch");
    c.N = (int64_t)c.n[0] * c.n[1] * c.n[2];
    c.c64.alloc(sizeof(double) * 5 * c.N);
    c.c32.alloc(sizeof(float) * 5 * c.N);
    launch(ctx, mg_coarsen, dim3((unsigned)((c.N + 255) / 256)), dim3(256), 0, geo_of(f), geo_of(c),
           f.c64.as<double>(), c.c64.as<double>());
    h->lv.push_back(std::move(c));
  }
  for (auto& l : h->lv) {
    launch(ctx, mg_to_f32, dim3((unsigned)((5 * l.N + 255) / 256)), dim3(256), 0, 5 * l.N, l.c64.as<double>(),
           l.c32.as<float>());
    l.di64.alloc(sizeof(double) * l.N);
    l.di32.alloc(sizeof(float) * l.N);
  }
  BKTS_HIP(hipGetLastError());
  ctx->sync();
  BKTS_REQUIRE(h->lv.back().N <= kCoarsestMax, "multigrid: coarsest level too large");
  return h.release();
}

void mg_vcycle(bkts_ctx ctx, const bkts_op_s& op, int dtype, int k, double a, double b, const void* F, void* Z) {
  BKTS_REQUIRE(k >= 1 && k <= BKTS_MAX_K, "k out of range");
  if (!op.mg) op.mg.reset(mg_build(const_cast<bkts_op>(&op)), mg_hier_delete);
  MgHier& h = *op.mg;
  if (h.a != a || h.b != b) {  // inverse diagonals of every level for this (a, b)
    for (auto& l : h.lv)
      launch(ctx, mg_dinv, dim3((unsigned)((l.N + 255) / 256)), dim3(256), 0, l.N, l.c64.as<double>(), a, b,
             l.di64.as<double>(), l.di32.as<float>());
    h.a = a;
    h.b = b;
  }
  if (dtype == BKTS_F64)
    vcycle<double>(ctx, *op.mg, 0, k, a, b, static_cast<const double*>(F), static_cast<double*>(Z));
  else
    vcycle<float>(ctx, *op.mg, 0, k, a, b, static_cast<const float*>(F), static_cast<float*>(Z));
  BKTS_HIP(hipGetLastError());
}

}  // namespace bkts

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
//   z = x + s P x_{l+1};  z += w D^-1 (f - A z)   (prolongation and post-sweep, one pass)
// with the pre-smoothed x recomputed wherever it is needed instead of stored, and on the coarsest
// level (at most 64 cells) a fixed number of damped Jacobi sweeps.  The scale s > 1 compensates the
// Galerkin operator of piecewise-constant aggregation, which is too stiff on smooth modes (an
// aggregate couples to a face neighbour through four fine faces), so an unscaled correction falls
// short.
//
// Launch structure.  The large levels run one multi-workgroup launch per restriction and per
// prolongation, each workgroup on a contiguous range of the grid that belongs to one XCD (so the
// neighbour lines and planes that a cell's stencil re-reads sit in that XCD's L2).  Every level
// whose block has at most kTailElems entries, down to the coarsest solve and back up, runs in ONE
// single-workgroup launch (the tail): its passes are separated by workgroup barriers instead of
// kernel boundaries; on the coarsest level the iterate lives in LDS and each thread keeps its
// elements' couplings in registers across the sweeps.  The finest
// prolongation can also fold the block-CG reductions that follow the preconditioner
// (gamma = R^T Z, T = Q^T Z and the column norms of R), since it already holds R and Z per row.
#include <limits>
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
constexpr double kOmega = 0.9;        // damping of the pre- and post-sweeps
constexpr double kCoarseScale = 1.4;  // scale of the prolonged coarse correction
constexpr double kCoarseOmega = 0.8;  // damping of the coarsest level's sweeps
constexpr int kMaxLevels = 16;
constexpr int64_t kTailElems = 2048;  // levels with N_l * k <= this run inside the tail launch
constexpr int kTailThreads = 512;

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
  T gc;  // scale of the prolonged coarse correction
  int k;
};

// CW consecutive values of one row as one vector access (one address per lane instead of CW; a row
// chunk starts at a multiple of CW elements and the blocks are 16-byte aligned).
template <typename T, int CW>
__device__ __forceinline__ void ld_cw(const T* p, T (&v)[CW]) {
  if constexpr (CW == 4 && sizeof(T) == 4) {
    const float4 q = *reinterpret_cast<const float4*>(p);
    v[0] = q.x; v[1] = q.y; v[2] = q.z; v[3] = q.w;
  } else if constexpr (CW == 2 && sizeof(T) == 4) {
    const float2 q = *reinterpret_cast<const float2*>(p);
    v[0] = q.x; v[1] = q.y;
  } else if constexpr (CW == 4 && sizeof(T) == 8) {
    const double2 a = *reinterpret_cast<const double2*>(p);
    const double2 b = *reinterpret_cast<const double2*>(p + 2);
    v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y;
  } else if constexpr (CW == 2 && sizeof(T) == 8) {
    const double2 a = *reinterpret_cast<const double2*>(p);
    v[0] = a.x; v[1] = a.y;
  } else {
#pragma unroll
    for (int j = 0; j < CW; ++j) v[j] = p[j];
  }
}

template <typename T, int CW>
__device__ __forceinline__ void st_cw(T* p, const T (&v)[CW]) {
  if constexpr (CW == 4 && sizeof(T) == 4) {
    *reinterpret_cast<float4*>(p) = float4{v[0], v[1], v[2], v[3]};
  } else if constexpr (CW == 2 && sizeof(T) == 4) {
    *reinterpret_cast<float2*>(p) = float2{v[0], v[1]};
  } else if constexpr (CW == 4 && sizeof(T) == 8) {
    *reinterpret_cast<double2*>(p) = double2{v[0], v[1]};
    *reinterpret_cast<double2*>(p + 2) = double2{v[2], v[3]};
  } else if constexpr (CW == 2 && sizeof(T) == 8) {
    *reinterpret_cast<double2*>(p) = double2{v[0], v[1]};
  } else {
#pragma unroll
    for (int j = 0; j < CW; ++j) p[j] = v[j];
  }
}

// Streaming load of rows that are dead after this kernel (Q in the finest prolongation): marked
// non-temporal, so they do not displace the f rows that the neighbouring planes re-read from L2.
// (Z is not streamed this way: the direction update reads it next, from the caches.)
template <typename T, int CW>
__device__ __forceinline__ void ld_cw_nt(const T* p, T (&v)[CW]) {
  if constexpr (CW == 4 && sizeof(T) == 4) {
    typedef float f4 __attribute__((ext_vector_type(4)));
    const f4 q = __builtin_nontemporal_load(reinterpret_cast<const f4*>(p));
    v[0] = q.x; v[1] = q.y; v[2] = q.z; v[3] = q.w;
  } else {
#pragma unroll
    for (int j = 0; j < CW; ++j) v[j] = __builtin_nontemporal_load(p + j);
  }
}

// Damped Jacobi from zero: x[r] = w f[r] / dA[r], for the CW columns starting at c0.
template <typename T, int CW>
__device__ __forceinline__ void pre_x(const LvArgs<T>& L, const T* f, int64_t r, int c0, T (&x)[CW]) {
  const T s = L.w * L.di[r];
  T fv[CW];
  ld_cw<T, CW>(f + r * L.k + c0, fv);
#pragma unroll
  for (int j = 0; j < CW; ++j) x[j] = s * fv[j];
}

// (A y)[r] for the CW columns at c0, where y at cell q = (qx, qy, qz) is produced by
// ycell(q, qx, qy, qz, out[CW]).  Neighbours in the order +x, -x, +y, -y, +z, -z.  Branch-free: an
// absent neighbour (grid boundary) is read at the cell itself with a zero coefficient, so the loads
// of all six neighbours are in flight together.
template <typename T, int CW, typename Y>
__device__ __forceinline__ void apply_row(const LvArgs<T>& L, int64_t r, int ix, int iy, int iz, const T (&yr)[CW],
                                          Y ycell, T (&out)[CW]) {
  const Geo& g = L.g;
  const int64_t N = g.N;
  const int pos[3] = {ix, iy, iz};
  const int len[3] = {g.nx, g.ny, g.nz};
  const int64_t st[3] = {g.sx, g.sy, g.sz};
  T cf[6];
  T y[6][CW];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const T* od = L.c + (2 + d) * N;
    const bool up = pos[d] + 1 < len[d], lo = pos[d] > 0;
    const int64_t ql = lo ? r - st[d] : r;
    // both couplings read unconditionally (a select on the loaded value would become a branch)
    cf[2 * d] = L.b * od[r] * T(up ? 1 : 0);
    cf[2 * d + 1] = L.b * od[ql] * T(lo ? 1 : 0);
    const int du = up ? 1 : 0, dl = lo ? 1 : 0;
    ycell(up ? r + st[d] : r, ix + (d == 0 ? du : 0), iy + (d == 1 ? du : 0), iz + (d == 2 ? du : 0), y[2 * d]);
    ycell(ql, ix - (d == 0 ? dl : 0), iy - (d == 1 ? dl : 0), iz - (d == 2 ? dl : 0), y[2 * d + 1]);
  }
  const T dA = T(1) / L.di[r];  // the diagonal from its cached inverse: no dK or mass read
#pragma unroll
  for (int j = 0; j < CW; ++j) out[j] = dA * yr[j];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
#pragma unroll
    for (int j = 0; j < CW; ++j) out[j] = fma(cf[2 * d], y[2 * d][j], out[j]);
#pragma unroll
    for (int j = 0; j < CW; ++j) out[j] = fma(cf[2 * d + 1], y[2 * d + 1][j], out[j]);
  }
}

// r = f - A x at fine cell i with x = w D^-1 f (the pre-smoothed iterate, recomputed from f).
template <typename T, int CW>
__device__ __forceinline__ void smoothed_residual(const LvArgs<T>& L, const T* f, int64_t i, int ix, int iy, int iz,
                                                  int c0, T (&v)[CW]) {
  T fi[CW], xi[CW], ax[CW];
  ld_cw<T, CW>(f + i * L.k + c0, fi);
  const T s = L.w * L.di[i];
#pragma unroll
  for (int j = 0; j < CW; ++j) xi[j] = s * fi[j];
  apply_row<T, CW>(L, i, ix, iy, iz, xi,
                   [&](int64_t q, int, int, int, T(&yq)[CW]) { pre_x<T, CW>(L, f, q, c0, yq); }, ax);
#pragma unroll
  for (int j = 0; j < CW; ++j) v[j] = fi[j] - ax[j];
}

// z = y + w D^-1 (f - A y) at fine cell r with y = w D^-1 f + P xc (coarse level c); also returns the
// row's f values.
// A cell's six neighbours lie in at most four aggregates: its own, and along each axis the one on
// the side where the cell is the outer child. Those four coarse values are loaded once and each
// neighbour takes its aggregate's.
template <typename T, int CW>
__device__ __forceinline__ void prolong_row(const LvArgs<T>& L, const Geo& c, const T* f, const T* xc, int64_t r,
                                            int ix, int iy, int iz, int c0, T (&zr)[CW], T (&fr)[CW]) {
  const int pos[3] = {ix, iy, iz};
  const int len[3] = {L.g.nx, L.g.ny, L.g.nz};
  const int64_t cst[3] = {1, c.sy, c.sz};
  const int64_t P0 = (ix >> 1) + c.sy * (iy >> 1) + c.sz * (iz >> 1);
  T xv[CW], xo[3][CW];
  ld_cw<T, CW>(xc + P0 * L.k + c0, xv);
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const bool odd = pos[d] & 1;
    const int po = odd ? pos[d] + 1 : pos[d] - 1;  // the neighbour outside the own aggregate
    const int64_t Po = (po >= 0 && po < len[d]) ? (odd ? P0 + cst[d] : P0 - cst[d]) : P0;
    ld_cw<T, CW>(xc + Po * L.k + c0, xo[d]);
  }
#pragma unroll
  for (int j = 0; j < CW; ++j) {
    xv[j] *= L.gc;
#pragma unroll
    for (int d = 0; d < 3; ++d) xo[d][j] *= L.gc;
  }
  auto ycell = [&](int64_t q, int qx, int qy, int qz, T(&y)[CW]) {
    pre_x<T, CW>(L, f, q, c0, y);
    const bool ox = (qx >> 1) != (ix >> 1), oy = (qy >> 1) != (iy >> 1), oz = (qz >> 1) != (iz >> 1);
#pragma unroll
    for (int j = 0; j < CW; ++j) y[j] += ox ? xo[0][j] : (oy ? xo[1][j] : (oz ? xo[2][j] : xv[j]));
  };
  T yr[CW], ay[CW];
  ld_cw<T, CW>(f + r * L.k + c0, fr);
  const T s = L.w * L.di[r];
#pragma unroll
  for (int j = 0; j < CW; ++j) yr[j] = s * fr[j] + xv[j];
  apply_row<T, CW>(L, r, ix, iy, iz, yr, ycell, ay);
#pragma unroll
  for (int j = 0; j < CW; ++j) zr[j] = yr[j] + s * (fr[j] - ay[j]);
}

// fc = P^T (f - A x) with x = w D^-1 f.  A workgroup covers a strip of 32 coarse cells along x: its
// 256 threads are the 64 x 2 x 2 fine cells of those aggregates (consecutive threads on consecutive
// cells of one grid line), each forms its own residual, and the 8 residuals of an aggregate are
// summed through LDS in a fixed order.  One-dimensional grid of gx * ncy * ncz strips, x fastest,
// remapped so that each XCD takes one contiguous range of strips.
template <typename T, int CW, bool FLAT>
__global__ __launch_bounds__(256) void mg_restrict_kernel(LvArgs<T> L, Geo c, int gx, const T* __restrict__ f,
                                                          T* __restrict__ fc) {
  __shared__ T red[CW][256];
  const int t = threadIdx.x;
  // 3-D: the 64 x 2 x 2 fine cells of 32 aggregates; FLAT (one cell along z): 64 x 4 cells, the 32 x 2
  // aggregates of two coarse rows, so no thread sits on the absent second z layer
  const int x = t & 63, y = FLAT ? (t >> 6) : ((t >> 6) & 1), z = FLAT ? 0 : (t >> 7);
  const int64_t unit = dev::xcd_slot(blockIdx.x, gridDim.x);
  const int64_t yz = unit / gx;
  const int X0 = (int)(unit - yz * gx) * 32;
  const int Y = FLAT ? 2 * (int)yz : (int)(yz % c.ny), Z = FLAT ? 0 : (int)(yz / c.ny);
  const Geo& g = L.g;
  const int ix = 2 * X0 + x, iy = 2 * Y + y, iz = 2 * Z + z;
  const bool in = ix < g.nx && iy < g.ny && iz < g.nz;
  const int64_t i = in ? ix + g.sy * iy + g.sz * iz : 0;
  for (int c0 = 0; c0 < L.k; c0 += CW) {
    T v[CW];
#pragma unroll
    for (int j = 0; j < CW; ++j) v[j] = T(0);
    if (in) smoothed_residual<T, CW>(L, f, i, ix, iy, iz, c0, v);
#pragma unroll
    for (int j = 0; j < CW; ++j) red[j][t] = v[j];
    __syncthreads();
    if (FLAT) {  // 64 aggregates: two coarse rows of 32, four children each, in the order of the 3-D sum
      const int ta = t & 31, tb = t >> 5;
      if (t < 64 && X0 + ta < c.nx && Y + tb < c.ny) {
        const int64_t R = (X0 + ta) + c.sy * (Y + tb);
#pragma unroll
        for (int j = 0; j < CW; ++j) {
          T sum = T(0);
#pragma unroll
          for (int q = 0; q < 4; ++q) sum += red[j][(2 * ta + (q & 1)) + 64 * (2 * tb + (q >> 1))];
          fc[R * L.k + c0 + j] = sum;
        }
      }
    } else if (t < 32 && X0 + t < c.nx) {
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

// z = y + w D^-1 (f - A y) with y = w D^-1 f + P xc.  Persistent: each workgroup walks one contiguous
// XCD-aware range of rows, one row per thread per step.  With GRAM (CW == k, k in {1, 2, 4}) the
// workgroup also accumulates gamma = f^T z, T = Q^T z and nrm = diag(f^T f) (per thread in the
// block's precision, then in FP64) and stores one partial per entry, laid out
// [gamma (k*k) | T (k*k) | nrm (k)] x gridDim.x (fixed-order folding).
template <typename T, int CW, bool GRAM>
__global__ __launch_bounds__(256) void mg_prolong_kernel(LvArgs<T> L, Geo c, const T* __restrict__ f,
                                                         const T* __restrict__ xc, T* __restrict__ z,
                                                         const T* __restrict__ Qm, double* partials) {
  constexpr int NA = GRAM ? 2 * CW * CW + CW : 1;
  // a thread's rows are summed in the block's own precision (FP32 blocks: about 16 rows per thread,
  // which keeps the accumulators in half the registers), the threads and workgroups in FP64
  using A = T;
  A acc[NA];
#pragma unroll
  for (int e = 0; e < NA; ++e) acc[e] = A(0);
  const int64_t N = L.g.N;
  const int64_t slot = dev::xcd_slot(blockIdx.x, gridDim.x);
  const dev::ChunkWalk walk = dev::xcd_chunks((N + 255) / 256);
  for (int64_t ch = walk.first; ch < walk.end; ch += walk.step) {
    const int64_t r = ch * 256 + threadIdx.x;
    if (r >= N) continue;  // the last chunk's tail
    int ix, iy, iz;
    coords(L.g, r, ix, iy, iz);
    const int kc = GRAM ? CW : L.k;  // with the reductions the row is one chunk
    for (int c0 = 0; c0 < kc; c0 += CW) {
      T zr[CW], fr[CW];
      prolong_row<T, CW>(L, c, f, xc, r, ix, iy, iz, c0, zr, fr);
      st_cw<T, CW>(z + r * L.k + c0, zr);
      if constexpr (GRAM) {
        T q[CW];
        ld_cw_nt<T, CW>(Qm + r * CW, q);
#pragma unroll
        for (int i = 0; i < CW; ++i) {
#pragma unroll
          for (int j = 0; j < CW; ++j) {
            acc[i * CW + j] = fma(fr[i], zr[j], acc[i * CW + j]);
            acc[CW * CW + i * CW + j] = fma(q[i], zr[j], acc[CW * CW + i * CW + j]);
          }
          acc[2 * CW * CW + i] = fma(fr[i], fr[i], acc[2 * CW * CW + i]);
        }
      }
    }
  }
  if constexpr (GRAM) {
    __shared__ double red[4 * NA];
    double sum[NA];
#pragma unroll
    for (int e = 0; e < NA; ++e) sum[e] = (double)acc[e];
#pragma unroll
    for (int off = 1; off < 64; off <<= 1)
#pragma unroll
      for (int e = 0; e < NA; ++e) sum[e] += __shfl_xor(sum[e], off);
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0) {
#pragma unroll
      for (int e = 0; e < NA; ++e) red[w * NA + e] = sum[e];
    }
    __syncthreads();
    for (int e = threadIdx.x; e < NA; e += 256)
      partials[(int64_t)e * gridDim.x + slot] = ((red[e] + red[NA + e]) + red[2 * NA + e]) + red[3 * NA + e];
  }
}

// The levels of the tail, finest first: the coefficients, the inverse diagonal, the right-hand side
// f and the output z (also the scratch of the level's residuals while restricting).
template <typename T>
struct TailLv {
  Geo g;
  const T* c;
  const T* di;
  T* f;
  T* z;
};

template <typename T>
struct TailArgs {
  TailLv<T> lv[kMaxLevels];
  int nl;  // levels in the tail; the last is the coarsest
  int k;
  T a, b, w, gc;
  T wc;  // damping of the coarsest level's sweeps
};

template <typename T>
__device__ __forceinline__ LvArgs<T> tail_lv(const TailArgs<T>& A, int l) {
  LvArgs<T> L;
  L.g = A.lv[l].g;
  L.c = A.lv[l].c;
  L.di = A.lv[l].di;
  L.a = A.a;
  L.b = A.b;
  L.w = A.w;
  L.gc = A.gc;
  L.k = A.k;
  return L;
}

// The tail of the V-cycle in one workgroup: for every tail level but the coarsest, the smoothed
// residual of each cell (into the level's z buffer) and then the aggregate sums into the next
// level's f; on the coarsest level kCoarseSweeps damped Jacobi sweeps with the coefficients and the
// iterate in LDS; then the prolongations and post-sweeps back up to the first tail level.  Each pass
// ends with a workgroup barrier, which also orders the global-memory hand-over between passes (all
// waves share one CU).  Sums over an aggregate run over its children in the same fixed order as the
// multi-workgroup restriction.
template <typename T, int CW>
__global__ __launch_bounds__(kTailThreads) void mg_tail_kernel(TailArgs<T> A) {
  __shared__ T xs[2][kCoarsestMax * BKTS_MAX_K];
  const int t = threadIdx.x;
  const int k = A.k;
  const int nch = k / CW;
  for (int l = 0; l + 1 < A.nl; ++l) {
    const LvArgs<T> L = tail_lv(A, l);
    const T* f = A.lv[l].f;
    T* s = A.lv[l].z;
    const int64_t n = L.g.N * nch;
    for (int64_t e = t; e < n; e += kTailThreads) {
      const int64_t i = e / nch;
      const int c0 = (int)(e - i * nch) * CW;
      int ix, iy, iz;
      coords(L.g, i, ix, iy, iz);
      T v[CW];
      smoothed_residual<T, CW>(L, f, i, ix, iy, iz, c0, v);
      st_cw<T, CW>(s + i * k + c0, v);
    }
    __syncthreads();
    const Geo g = L.g, gc = A.lv[l + 1].g;
    T* fc = A.lv[l + 1].f;
    const int64_t nc = gc.N * nch;
    for (int64_t e = t; e < nc; e += kTailThreads) {
      const int64_t R = e / nch;
      const int c0 = (int)(e - R * nch) * CW;
      int X, Y, Z;
      coords(gc, R, X, Y, Z);
      T sum[CW];
#pragma unroll
      for (int j = 0; j < CW; ++j) sum[j] = T(0);
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int ix = 2 * X + (q & 1), iy = 2 * Y + ((q >> 1) & 1), iz = 2 * Z + (q >> 2);
        if (ix < g.nx && iy < g.ny && iz < g.nz) {
          T v[CW];
          ld_cw<T, CW>(s + (ix + g.sy * iy + g.sz * iz) * k + c0, v);
#pragma unroll
          for (int j = 0; j < CW; ++j) sum[j] += v[j];
        }
      }
      st_cw<T, CW>(fc + R * k + c0, sum);
    }
    __syncthreads();
  }
  {  // coarsest level: each thread keeps its elements' neighbour indices and coefficients in
     // registers for all sweeps, and only the iterate moves through LDS
    constexpr int kCE = (kCoarsestMax * BKTS_MAX_K + kTailThreads - 1) / kTailThreads;
    const int l = A.nl - 1;
    const LvArgs<T> L = tail_lv(A, l);
    const Geo& g = L.g;
    const int n = (int)(g.N * k);
    const T* f = A.lv[l].f;
    int nb[kCE][6];
    T cf[kCE][6], fv[kCE], dA[kCE], di[kCE];
#pragma unroll
    for (int i = 0; i < kCE; ++i) {
      const int e = t + i * kTailThreads;
      if (e < n) {
        const int r = e / k, col = e - r * k;
        int ix, iy, iz;
        coords(g, r, ix, iy, iz);
        const int pos[3] = {ix, iy, iz};
        const int len[3] = {g.nx, g.ny, g.nz};
        const int st[3] = {1, g.nx, g.nx * g.ny};
#pragma unroll
        for (int d = 0; d < 3; ++d) {  // same neighbour order and zero-coefficient rule as apply_row
          const T* od = L.c + (2 + d) * g.N;
          const bool up = pos[d] + 1 < len[d], lo = pos[d] > 0;
          const int ql = lo ? r - st[d] : r;
          nb[i][2 * d] = (up ? r + st[d] : r) * k + col;
          nb[i][2 * d + 1] = ql * k + col;
          cf[i][2 * d] = L.b * od[r] * T(up ? 1 : 0);
          cf[i][2 * d + 1] = L.b * od[ql] * T(lo ? 1 : 0);
        }
        di[i] = L.di[r];
        dA[i] = T(1) / di[i];
        fv[i] = f[e];
        xs[0][e] = A.wc * fv[i] * di[i];
      }
    }
    __syncthreads();
    int cur = 0;
    for (int it = 1; it < kCoarseSweeps; ++it) {
#pragma unroll
      for (int i = 0; i < kCE; ++i) {
        const int e = t + i * kTailThreads;
        if (e < n) {
          const T yr = xs[cur][e];
          T ay = dA[i] * yr;
#pragma unroll
          for (int q = 0; q < 6; ++q) ay = fma(cf[i][q], xs[cur][nb[i][q]], ay);
          xs[cur ^ 1][e] = yr + A.wc * (fv[i] - ay) * di[i];
        }
      }
      __syncthreads();
      cur ^= 1;
    }
    T* z = A.lv[l].z;
    for (int e = t; e < n; e += kTailThreads) z[e] = xs[cur][e];
    __syncthreads();
  }
  for (int l = A.nl - 2; l >= 0; --l) {
    const LvArgs<T> L = tail_lv(A, l);
    const Geo gc = A.lv[l + 1].g;
    const T* f = A.lv[l].f;
    const T* xc = A.lv[l + 1].z;
    T* z = A.lv[l].z;
    const int64_t n = L.g.N * nch;
    for (int64_t e = t; e < n; e += kTailThreads) {
      const int64_t i = e / nch;
      const int c0 = (int)(e - i * nch) * CW;
      int ix, iy, iz;
      coords(L.g, i, ix, iy, iz);
      T zr[CW], fr[CW];
      prolong_row<T, CW>(L, gc, f, xc, i, ix, iy, iz, c0, zr, fr);
      st_cw<T, CW>(z + i * k + c0, zr);
    }
    __syncthreads();
  }
}

// First level of the tail for block width k.
int tail_start(const MgHier& h, int k) {
  const int nl = (int)h.lv.size();
  int t0 = 0;
  while (t0 + 1 < nl && h.lv[t0].N * k > kTailElems) ++t0;
  return t0;
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
  L.gc = (T)kCoarseScale;
  L.k = k;
  return L;
}

// Persistent grid of the prolongation: the resident capacity of the chip, capped by the row chunks,
// in whole rounds over the XCDs when it has at least one.
template <typename K>
int64_t prolong_grid(bkts_ctx ctx, K kernel, int64_t N) {
  int64_t nb = (int64_t)blocks_per_cu(reinterpret_cast<const void*>(kernel)) * ctx->num_cu;
  const int64_t chunks = (N + 255) / 256;
  if (nb > chunks) nb = chunks;
  if (nb >= dev::kXcd) nb -= nb % dev::kXcd;
  return nb < 1 ? 1 : nb;
}

template <typename T, int CW, bool GRAM>
void launch_prolong(bkts_ctx ctx, const LvArgs<T>& L, const Geo& gc, const T* f, const T* xc, T* z, const T* Q,
                    double* partials, int64_t nb) {
  launch(ctx, (mg_prolong_kernel<T, CW, GRAM>), dim3((unsigned)nb), dim3(256), 0, L, gc, f, xc, z, Q, partials);
}

template <typename T, int CW, bool GRAM>
void prolong_level(bkts_ctx ctx, const LvArgs<T>& L, const Geo& gc, const T* f, const T* xc, T* z) {
  const int64_t nb = prolong_grid(ctx, mg_prolong_kernel<T, CW, GRAM>, L.g.N);
  launch_prolong<T, CW, GRAM>(ctx, L, gc, f, xc, z, nullptr, nullptr, nb);
}

// Finest prolongation with the fused reductions: partials of NA = 2k^2 + k entries per workgroup.
template <typename T, int CW>
void prolong_fused(bkts_ctx ctx, const LvArgs<T>& L, const Geo& gc, const T* f, const T* xc, T* z, MgFuse* fuse,
                   const std::string& tag) {
  const int64_t nb = prolong_grid(ctx, mg_prolong_kernel<T, CW, true>, L.g.N);
  double* part = ctx->ws.get<double>("mg_fuse_part" + tag, (size_t)(2 * CW * CW + CW) * nb);
  launch_prolong<T, CW, true>(ctx, L, gc, f, xc, z, static_cast<const T*>(fuse->Q), part, nb);
  fuse->partials = part;
  fuse->nslots = nb;
}

template <typename T>
void vcycle(bkts_ctx ctx, MgHier& h, int k, double a, double b, const T* f, T* z, MgFuse* fuse) {
  const int nl = (int)h.lv.size();
  const double sv = sizeof(T);
  const std::string tag = sizeof(T) == 8 ? "d" : "s";
  // per-level right-hand sides and iterates: the caller's F and Z on level 0, workspace below
  std::vector<T*> fb(nl), zb(nl);
  fb[0] = const_cast<T*>(f);
  zb[0] = z;
  for (int l = 1; l < nl; ++l) {
    fb[l] = ctx->ws.get<T>("mg_f" + std::to_string(l) + tag, (size_t)h.lv[l].N * k);
    zb[l] = ctx->ws.get<T>("mg_x" + std::to_string(l) + tag, (size_t)h.lv[l].N * k);
  }
  const int t0 = tail_start(h, k);
  const int cw = chunk_width(k);
  for (int l = 0; l < t0; ++l) {
    const MgLevel& lf = h.lv[l];
    const MgLevel& lc = h.lv[l + 1];
    const LvArgs<T> L = lv_args<T>(lf, k, a, b);
    const Geo gc = geo_of(lc);
    const int gx = (lc.n[0] + 31) / 32;
    const bool flat = lf.n[2] == 1;  // 2-D (or 1-D) level: strips of two coarse rows
    const int64_t nbr = flat ? (int64_t)gx * ((lc.n[1] + 1) / 2) : (int64_t)gx * lc.n[1] * lc.n[2];
    BKTS_REQUIRE(nbr < ((int64_t)1 << 31), "multigrid: grid too large for the restriction launch");
    // algorithmic bytes: f, the inverse diagonal and the 3 coupling arrays read, the coarse f written
    ProfScope prof(ctx, l == 0 ? BKTS_K_MG_RESTRICT : BKTS_K_MG_COARSE,
                   sv * (1.0 * lf.N * k + 4.0 * lf.N + 1.0 * lc.N * k));
    const dim3 gr((unsigned)nbr);
    auto go = [&](auto kernel) { launch(ctx, kernel, gr, dim3(256), 0, L, gc, gx, (const T*)fb[l], fb[l + 1]); };
    if (cw == 4)
      flat ? go(mg_restrict_kernel<T, 4, true>) : go(mg_restrict_kernel<T, 4, false>);
    else if (cw == 2)
      flat ? go(mg_restrict_kernel<T, 2, true>) : go(mg_restrict_kernel<T, 2, false>);
    else
      flat ? go(mg_restrict_kernel<T, 1, true>) : go(mg_restrict_kernel<T, 1, false>);
  }
  {
    TailArgs<T> A{};
    A.nl = nl - t0;
    A.k = k;
    A.a = (T)a;
    A.b = (T)b;
    A.w = (T)kOmega;
    A.gc = (T)kCoarseScale;
    A.wc = (T)kCoarseOmega;
    double bytes = 0.0;
    for (int l = t0; l < nl; ++l) {
      const LvArgs<T> L = lv_args<T>(h.lv[l], k, a, b);
      TailLv<T>& tl = A.lv[l - t0];
      tl.g = L.g;
      tl.c = L.c;
      tl.di = L.di;
      tl.f = fb[l];
      tl.z = zb[l];
      bytes += sv * (2.0 * h.lv[l].N * k + 4.0 * h.lv[l].N);
    }
    ProfScope prof(ctx, BKTS_K_MG_COARSE, bytes);
    if (cw == 4)
      launch(ctx, (mg_tail_kernel<T, 4>), dim3(1), dim3(kTailThreads), 0, A);
    else if (cw == 2)
      launch(ctx, (mg_tail_kernel<T, 2>), dim3(1), dim3(kTailThreads), 0, A);
    else
      launch(ctx, (mg_tail_kernel<T, 1>), dim3(1), dim3(kTailThreads), 0, A);
  }
  const bool gram = fuse && t0 >= 1 && (k == 1 || k == 2 || k == 4);
  if (fuse) fuse->nslots = 0;
  for (int l = t0 - 1; l >= 0; --l) {
    const MgLevel& lf = h.lv[l];
    const MgLevel& lc = h.lv[l + 1];
    const LvArgs<T> L = lv_args<T>(lf, k, a, b);
    const Geo gc = geo_of(lc);
    const T* fl = fb[l];
    const T* xc = zb[l + 1];
    T* zl = zb[l];
    // algorithmic bytes: f, the coarse x, the inverse diagonal and the 3 coupling arrays read, z
    // written (and Q read when the reductions are fused)
    const bool g = gram && l == 0;
    const bool q_own = g && fuse->Q != static_cast<const void*>(fl);  // Q = f is read once
    ProfScope prof(ctx, l == 0 ? BKTS_K_MG_PROLONG : BKTS_K_MG_COARSE,
                   sv * ((q_own ? 3.0 : 2.0) * lf.N * k + 4.0 * lf.N + 1.0 * lc.N * k));
    if (g) {
      if (k == 4)
        prolong_fused<T, 4>(ctx, L, gc, fl, xc, zl, fuse, tag);
      else if (k == 2)
        prolong_fused<T, 2>(ctx, L, gc, fl, xc, zl, fuse, tag);
      else
        prolong_fused<T, 1>(ctx, L, gc, fl, xc, zl, fuse, tag);
    } else if (cw == 4) {
      prolong_level<T, 4, false>(ctx, L, gc, fl, xc, zl);
    } else if (cw == 2) {
      prolong_level<T, 2, false>(ctx, L, gc, fl, xc, zl);
    } else {
      prolong_level<T, 1, false>(ctx, L, gc, fl, xc, zl);
    }
  }
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
  while (h->lv.back().N > kCoarsestMax && (int)h->lv.size() < kMaxLevels) {
    const MgLevel& f = h->lv.back();
    MgLevel c;
    for (int d = 0; d < 3; ++d) c.n[d] = (f.n[d] + 1) / 2;
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

// Level 0 and the Galerkin products of every coarser level from the operator's current stencil
// values, into the buffers of an existing hierarchy; the inverse diagonals follow on the next cycle.
void mg_refresh(bkts_ctx ctx, const bkts_op_s& op) {
  if (!op.mg) return;
  MgHier& h = *op.mg;
  MgLevel& l0 = h.lv[0];
  int sel[3] = {-1, -1, -1};
  int64_t s = 1;
  for (int d = 0; d < 3; ++d) {
    if (l0.n[d] >= 2)
      for (int q = 0; q < op.st_na; ++q)
        if (op.st_off[q] == s) sel[d] = q;
    s *= l0.n[d];
  }
  launch(ctx, mg_level0, dim3((unsigned)((l0.N + 255) / 256)), dim3(256), 0, l0.N, op.st_na, op.st_coef.as<double>(),
         sel[0], sel[1], sel[2], l0.c64.as<double>());
  for (size_t l = 0; l + 1 < h.lv.size(); ++l) {
    const MgLevel& f = h.lv[l];
    MgLevel& c = h.lv[l + 1];
    launch(ctx, mg_coarsen, dim3((unsigned)((c.N + 255) / 256)), dim3(256), 0, geo_of(f), geo_of(c),
           f.c64.as<double>(), c.c64.as<double>());
  }
  for (auto& l : h.lv)
    launch(ctx, mg_to_f32, dim3((unsigned)((5 * l.N + 255) / 256)), dim3(256), 0, 5 * l.N, l.c64.as<double>(),
           l.c32.as<float>());
  BKTS_HIP(hipGetLastError());
  h.a = h.b = std::numeric_limits<double>::quiet_NaN();  // compares unequal: the next cycle recomputes
}

namespace {

// Stencil form of (J + J^T) / 2 from J's CSR rows (structurally symmetric stencil sparsity): the
// diagonal, then for each offset s the coupling to r + s, zero where r + s is not a neighbour.
__global__ void sym_stencil_kernel(int64_t N, int na, int64_t s0, int64_t s1, int64_t s2,
                                   const int32_t* __restrict__ rowptr, const int32_t* __restrict__ col,
                                   const double* __restrict__ val, double* __restrict__ st) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= N) return;
  const int64_t so[3] = {s0, s1, s2};
  double dg = 0.0, up[3] = {0.0, 0.0, 0.0};
  bool has[3] = {false, false, false};
  for (int32_t p = rowptr[r]; p < rowptr[r + 1]; ++p) {
    const int64_t c = col[p];
    if (c == r) dg = val[p];
    for (int q = 0; q < na; ++q)
      if (c == r + so[q]) {
        up[q] = val[p];
        has[q] = true;
      }
  }
  st[r] = dg;
  for (int q = 0; q < na; ++q) {
    double lo = 0.0;
    if (has[q]) {
      const int64_t rq = r + so[q];
      for (int32_t p = rowptr[rq]; p < rowptr[rq + 1]; ++p)
        if (col[p] == r) lo = val[p];
    }
    st[(int64_t)(1 + q) * N + r] = has[q] ? 0.5 * (up[q] + lo) : 0.0;
  }
}

}  // namespace

std::shared_ptr<bkts_op_s> sym_stencil_create(const bkts_op_s& J) {
  if (J.grid.dim < 1) return nullptr;
  auto S = std::make_shared<bkts_op_s>();
  S->ctx = J.ctx;
  S->N = J.N;
  S->grid = J.grid;
  S->format = BKTS_FMT_STENCIL;
  int64_t stride = 1;
  for (int d = 0; d < J.grid.dim; ++d) {
    if (J.grid.n[d] >= 2) S->st_off[S->st_na++] = stride;
    stride *= J.grid.n[d];
  }
  if (S->st_na == 0) return nullptr;
  S->st_coef.alloc(sizeof(double) * (1 + S->st_na) * J.N);
  return S;
}

void sym_stencil_refresh(bkts_ctx ctx, const bkts_op_s& J, bkts_op_s& S) {
  BKTS_REQUIRE(S.N == J.N && S.st_na > 0, "symmetric stencil form does not match its Jacobian");
  ProfScope prof(ctx, BKTS_K_OTHER, 12.0 * J.nnz * 2 + 8.0 * (1 + S.st_na) * J.N);
  launch(ctx, sym_stencil_kernel, dim3((unsigned)((J.N + 255) / 256)), dim3(256), 0, J.N, S.st_na, S.st_off[0],
         S.st_off[1], S.st_off[2], J.rowptr.as<int32_t>(), J.col.as<int32_t>(), J.val.as<double>(),
         S.st_coef.as<double>());
  BKTS_HIP(hipGetLastError());
}

const bkts_op_s* mg_source(bkts_ctx ctx, const bkts_op_s& op) {
  if (op.st_na > 0) return &op;
  if (!op.mg_sym) return nullptr;
  if (op.mg_sym_stale) {
    sym_stencil_refresh(ctx, op, *op.mg_sym);
    mg_refresh(ctx, *op.mg_sym);
    op.mg_sym_stale = false;
  }
  return op.mg_sym.get();
}

bool mg_fusable(bkts_ctx ctx, const bkts_op_s& op, int k) {
  (void)ctx;
  if (!(k == 1 || k == 2 || k == 4)) return false;
  if (!op.mg) op.mg.reset(mg_build(const_cast<bkts_op>(&op)), mg_hier_delete);
  return tail_start(*op.mg, k) >= 1;
}

void mg_vcycle(bkts_ctx ctx, const bkts_op_s& op, int dtype, int k, double a, double b, const void* F, void* Z,
               MgFuse* fuse) {
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
    vcycle<double>(ctx, h, k, a, b, static_cast<const double*>(F), static_cast<double*>(Z), fuse);
  else
    vcycle<float>(ctx, h, k, a, b, static_cast<const float*>(F), static_cast<float*>(Z), fuse);
  BKTS_HIP(hipGetLastError());
}

}  // namespace bkts

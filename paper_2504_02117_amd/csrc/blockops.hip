// Block-vector kernels on row tiles: Gram matrices X^T Y and column norms (FP64 accumulation,
// deterministic two-pass reduction), the fused block-CG updates with their Gram epilogues, the
// k x k right multiplication, scaled precision casts and small elementwise helpers.
//
// A tile is RT = 2048/KP rows of a block padded to KP columns.  Thread t owns column t % KP of
// eight rows, loads them with coalesced accesses and keeps them in registers; the tile is also
// staged in LDS so that a thread can read whole rows (for right multiplications by k x k
// matrices and for Gram accumulation).  Each persistent workgroup walks one contiguous range of
// tiles (XCD-aware) and leaves one partial k x k result; finalize_partials() folds the partials in
// a fixed order, so results are bitwise reproducible.
#include <map>
#include <mutex>

#include "devcommon.hpp"
#include "internal.hpp"
#include "wide.hpp"

namespace bkts {
namespace {

using dev::TileGeom;

template <int KP>
constexpr int lds_doubles(int ntiles) {
  return (ntiles * TileGeom<KP>::LDS_DOUBLES > 4 * KP * KP) ? ntiles * TileGeom<KP>::LDS_DOUBLES : 4 * KP * KP;
}

struct Slots {
  int64_t ntiles, nslots, tps;  // tiles, workgroups, tiles per workgroup
};

template <int KP>
Slots make_slots(bkts_ctx ctx, int64_t N) {
  Slots s;
  s.ntiles = (N + TileGeom<KP>::RT - 1) / TileGeom<KP>::RT;
  const int64_t cap = 2 * (int64_t)ctx->num_cu;
  s.nslots = s.ntiles < cap ? s.ntiles : cap;
  if (s.nslots < 1) s.nslots = 1;
  s.tps = (s.ntiles + s.nslots - 1) / s.nslots;
  return s;
}

// ---------------------------------------------------------------- Gram / norms

template <typename T, int KP>
__global__ __launch_bounds__(256) void gram_kernel(int64_t N, int k, const T* __restrict__ X, int ldx,
                                                   const T* __restrict__ Y, int ldy, double* partials,
                                                   int64_t tps) {
  using G = TileGeom<KP>;
  __shared__ __align__(16) double lds[lds_doubles<KP>(1)];
  const int t = threadIdx.x, c = t % KP, r0 = t / KP;
  const int64_t slot = dev::xcd_slot(blockIdx.x, gridDim.x);
  const int64_t ntiles = (N + G::RT - 1) / G::RT;
  double acc[KP];
#pragma unroll
  for (int a = 0; a < KP; ++a) acc[a] = 0.0;
  const int64_t tend = (slot + 1) * tps < ntiles ? (slot + 1) * tps : ntiles;
  for (int64_t tile = slot * tps; tile < tend; ++tile) {
    const int64_t row0 = tile * G::RT;
    double y[G::RPT];
#pragma unroll
    for (int i = 0; i < G::RPT; ++i) {
      const int row = r0 + i * G::RS;
      const int64_t gr = row0 + row;
      const bool ok = gr < N && c < k;
      lds[row * G::LDL + c] = ok ? dev::ld_d(X + gr * ldx + c) : 0.0;
      y[i] = ok ? dev::ld_d(Y + gr * ldy + c) : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < G::RPT; ++i) dev::lds_row_axpy<KP>(lds, r0 + i * G::RS, y[i], acc);
    __syncthreads();
  }
  dev::block_reduce_store<KP, KP>(acc, lds, partials, gridDim.x, slot);
}

template <typename T, int KP>
__global__ __launch_bounds__(256) void colnorm_kernel(int64_t N, int k, const T* __restrict__ X, int ldx,
                                                      double* partials, int64_t tps) {
  using G = TileGeom<KP>;
  __shared__ double red[4 * KP];
  const int t = threadIdx.x, c = t % KP, r0 = t / KP;
  const int64_t slot = dev::xcd_slot(blockIdx.x, gridDim.x);
  const int64_t ntiles = (N + G::RT - 1) / G::RT;
  double acc[1] = {0.0};
  const int64_t tend = (slot + 1) * tps < ntiles ? (slot + 1) * tps : ntiles;
  for (int64_t tile = slot * tps; tile < tend; ++tile) {
    const int64_t row0 = tile * G::RT;
#pragma unroll
    for (int i = 0; i < G::RPT; ++i) {
      const int64_t gr = row0 + r0 + i * G::RS;
      const double v = (gr < N && c < k) ? dev::ld_d(X + gr * ldx + c) : 0.0;
      acc[0] = fma(v, v, acc[0]);
    }
  }
  dev::block_reduce_store<KP, 1>(acc, red, partials, gridDim.x, slot);
}

// Column-wise dot products of up to three pairs of contiguous blocks (ld = k), FP64 accumulation:
// partial entry p*KP + c holds sum_r X_p[r][c] Y_p[r][c].
struct DotPairs {
  const void* x[3];
  const void* y[3];
};

template <typename T, int KP, int NP>
__global__ __launch_bounds__(256) void coldots_kernel(int64_t N, int k, DotPairs d, double* partials, int64_t tps) {
  using G = TileGeom<KP>;
  __shared__ double red[4 * NP * KP];
  const int t = threadIdx.x, c = t % KP, r0 = t / KP;
  const int64_t slot = dev::xcd_slot(blockIdx.x, gridDim.x);
  const int64_t ntiles = (N + G::RT - 1) / G::RT;
  double acc[NP];
#pragma unroll
  for (int p = 0; p < NP; ++p) acc[p] = 0.0;
  const int64_t tend = (slot + 1) * tps < ntiles ? (slot + 1) * tps : ntiles;
  for (int64_t tile = slot * tps; tile < tend; ++tile) {
    const int64_t row0 = tile * G::RT;
#pragma unroll
    for (int i = 0; i < G::RPT; ++i) {
      const int64_t gr = row0 + r0 + i * G::RS;
      if (gr < N && c < k) {
#pragma unroll
        for (int p = 0; p < NP; ++p)
          acc[p] = fma(dev::ld_d(static_cast<const T*>(d.x[p]) + gr * k + c),
                       dev::ld_d(static_cast<const T*>(d.y[p]) + gr * k + c), acc[p]);
      }
    }
  }
  dev::block_reduce_store<KP, NP>(acc, red, partials, gridDim.x, slot);
}

// Column-wise dot products for full-width, 16-byte aligned contiguous blocks (k == KP, rows of
// 16 bytes or more): each lane owns VEC = 16 / sizeof(T) consecutive columns of a row and loads them
// as one 16-byte vector, LPR = KP / VEC lanes share a row, and persistent workgroups (the resident
// capacity of the chip) walk contiguous XCD-aware row ranges.  FP64 accumulation; lanes with the
// same columns are summed by shuffles in a fixed order, then the four waves through LDS.  Same
// partial layout as coldots_kernel (entry p*KP + c).
template <typename T, int KP, int NP>
__global__ __launch_bounds__(256) void coldots_vec_kernel(int64_t N, DotPairs d, double* partials) {
  constexpr int VEC = 16 / sizeof(T);
  constexpr int LPR = KP / VEC;
  constexpr int RPW = 256 / LPR;  // rows per workgroup step
  typedef T vt __attribute__((ext_vector_type(VEC)));
  __shared__ double red[4][NP * KP];
  const int t = threadIdx.x, l = t % LPR;
  const int64_t slot = dev::xcd_slot(blockIdx.x, gridDim.x);
  const int64_t per = (N + gridDim.x - 1) / gridDim.x;
  const int64_t r_begin = slot * per, r_end = r_begin + per < N ? r_begin + per : N;
  double acc[NP][VEC];
#pragma unroll
  for (int p = 0; p < NP; ++p)
#pragma unroll
    for (int v = 0; v < VEC; ++v) acc[p][v] = 0.0;
  for (int64_t r = r_begin + t / LPR; r < r_end; r += RPW) {
    vt x[NP], y[NP];
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      x[p] = *reinterpret_cast<const vt*>(static_cast<const T*>(d.x[p]) + r * KP + l * VEC);
      y[p] = *reinterpret_cast<const vt*>(static_cast<const T*>(d.y[p]) + r * KP + l * VEC);
    }
#pragma unroll
    for (int p = 0; p < NP; ++p)
#pragma unroll
      for (int v = 0; v < VEC; ++v) acc[p][v] = fma((double)x[p][v], (double)y[p][v], acc[p][v]);
  }
#pragma unroll
  for (int off = LPR; off < 64; off <<= 1)
#pragma unroll
    for (int p = 0; p < NP; ++p)
#pragma unroll
      for (int v = 0; v < VEC; ++v) acc[p][v] += __shfl_xor(acc[p][v], off);
  const int w = t >> 6, lane = t & 63;
  if (lane < LPR) {
#pragma unroll
    for (int p = 0; p < NP; ++p)
#pragma unroll
      for (int v = 0; v < VEC; ++v) red[w][p * KP + lane * VEC + v] = acc[p][v];
  }
  __syncthreads();
  for (int e = t; e < NP * KP; e += 256)
    partials[(int64_t)e * gridDim.x + slot] = ((red[0][e] + red[1][e]) + red[2][e]) + red[3][e];
}

// out[i] = sum over slots of partials[e(i)][slot], e(i) = (i / kout) * KP + i % kout for the
// Gram layout (nrow = kout) or e(i) = i for vectors (nrow = 1).  One workgroup per output entry,
// fixed summation order.
__global__ __launch_bounds__(256) void finalize_kernel(const double* partials, int64_t nslots, int kout, int KPin,
                                                       int vector_mode, double* out) {
  __shared__ double s[256];
  const int i = blockIdx.x;
  const int e = vector_mode ? i : (i / kout) * KPin + i % kout;
  const double* p = partials + (int64_t)e * nslots;
  double acc = 0.0;
  for (int64_t j = threadIdx.x; j < nslots; j += 256) acc += p[j];
  s[threadIdx.x] = acc;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) s[threadIdx.x] += s[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[i] = s[0];
}

struct FoldArgs {
  FoldSet set[3];
  int nsets;
  int k;
  int64_t nslots;
};

// One workgroup per output entry of all sets (fixed summation order, as finalize_kernel).
__global__ __launch_bounds__(256) void finalize_sets_kernel(FoldArgs a) {
  __shared__ double s[256];
  int i = blockIdx.x, si = 0;
  for (; si < a.nsets; ++si) {
    const int E = a.set[si].vector ? a.k : a.k * a.k;
    if (i < E) break;
    i -= E;
  }
  const FoldSet& f = a.set[si];
  const int e = f.vector ? i : (i / a.k) * f.KP + i % a.k;
  const double* p = f.partials + (int64_t)e * a.nslots;
  double acc = 0.0;
  for (int64_t j = threadIdx.x; j < a.nslots; j += 256) acc += p[j];
  s[threadIdx.x] = acc;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) s[threadIdx.x] += s[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) f.out[i] = s[0];
}

// ---------------------------------------------------------------- block CG updates

// Load the k x k matrix M (row-major, device) column c into registers: col[j] = M[j][c].
template <int KP>
__device__ __forceinline__ void load_col(const double* M, int k, int c, double (&col)[KP]) {
#pragma unroll
  for (int j = 0; j < KP; ++j) col[j] = (j < k && c < k) ? M[j * k + c] : 0.0;
}

__device__ __forceinline__ double dinv_at(const double* dinv, int64_t r) { return dinv ? dinv[r] : 1.0; }

// X += P alpha; R -= Q alpha; Z = Dinv R; gamma = R^T Z; T = Q^T Z; nrm = diag(R^T R).
template <typename T, int KP>
__global__ __launch_bounds__(256) void cg_update_kernel(int64_t N, int k, T* __restrict__ X, const T* __restrict__ P,
                                                        T* __restrict__ R, const T* __restrict__ Q,
                                                        const double* __restrict__ alpha, const double* dinv,
                                                        double* pg, double* pt, double* pn, int64_t tps) {
  using G = TileGeom<KP>;
  __shared__ __align__(16) double lds[lds_doubles<KP>(2)];
  double* Pl = lds;
  double* Ql = lds + G::LDS_DOUBLES;
  const int t = threadIdx.x, c = t % KP, r0 = t / KP;
  const int64_t slot = dev::xcd_slot(blockIdx.x, gridDim.x);
  const int64_t ntiles = (N + G::RT - 1) / G::RT;
  double acol[KP];
  load_col<KP>(alpha, k, c, acol);
  double gacc[KP], tacc[KP], nacc[1] = {0.0};
#pragma unroll
  for (int a = 0; a < KP; ++a) gacc[a] = tacc[a] = 0.0;
  const int64_t tend = (slot + 1) * tps < ntiles ? (slot + 1) * tps : ntiles;
  for (int64_t tile = slot * tps; tile < tend; ++tile) {
    const int64_t row0 = tile * G::RT;
    double x[G::RPT], r[G::RPT], z[G::RPT];
#pragma unroll
    for (int i = 0; i < G::RPT; ++i) {
      const int row = r0 + i * G::RS;
      const int64_t gr = row0 + row;
      const bool ok = gr < N && c < k;
      const int64_t e = gr * k + c;
      Pl[row * G::LDL + c] = ok ? dev::ld_d(P + e) : 0.0;
      Ql[row * G::LDL + c] = ok ? dev::ld_d(Q + e) : 0.0;
      x[i] = ok ? dev::ld_d(X + e) : 0.0;
      r[i] = ok ? dev::ld_d(R + e) : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < G::RPT; ++i) {
      const int row = r0 + i * G::RS;
      const int64_t gr = row0 + row;
      x[i] += dev::lds_row_dot<KP>(Pl, row, acol);
      r[i] -= dev::lds_row_dot<KP>(Ql, row, acol);
      const bool ok = gr < N && c < k;
      z[i] = ok ? r[i] * dinv_at(dinv, gr) : 0.0;
      if (ok) {
        X[gr * k + c] = (T)x[i];
        R[gr * k + c] = (T)r[i];
      } else {
        r[i] = 0.0;
      }
      nacc[0] = fma(r[i], r[i], nacc[0]);
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < G::RPT; ++i) Pl[(r0 + i * G::RS) * G::LDL + c] = r[i];  // R tile replaces P tile
    __syncthreads();
#pragma unroll
    for (int i = 0; i < G::RPT; ++i) {
      const int row = r0 + i * G::RS;
      dev::lds_row_axpy<KP>(Pl, row, z[i], gacc);
      dev::lds_row_axpy<KP>(Ql, row, z[i], tacc);
    }
    __syncthreads();
  }
  dev::block_reduce_store<KP, KP>(gacc, lds, pg, gridDim.x, slot);
  dev::block_reduce_store<KP, KP>(tacc, lds, pt, gridDim.x, slot);
  dev::block_reduce_store<KP, 1>(nacc, lds, pn, gridDim.x, slot);
}

// P = Dinv R + P beta   (beta == nullptr: P = Dinv R)
template <typename T, int KP>
__global__ __launch_bounds__(256) void cg_pupdate_kernel(int64_t N, int k, T* __restrict__ P, const T* __restrict__ R,
                                                         const double* __restrict__ beta, const double* dinv,
                                                         int64_t tps) {
  using G = TileGeom<KP>;
  __shared__ __align__(16) double lds[lds_doubles<KP>(1)];
  const int t = threadIdx.x, c = t % KP, r0 = t / KP;
  const int64_t slot = dev::xcd_slot(blockIdx.x, gridDim.x);
  const int64_t ntiles = (N + G::RT - 1) / G::RT;
  double bcol[KP];
  if (beta) load_col<KP>(beta, k, c, bcol);
  const int64_t tend = (slot + 1) * tps < ntiles ? (slot + 1) * tps : ntiles;
  for (int64_t tile = slot * tps; tile < tend; ++tile) {
    const int64_t row0 = tile * G::RT;
    double r[G::RPT];
#pragma unroll
    for (int i = 0; i < G::RPT; ++i) {
      const int row = r0 + i * G::RS;
      const int64_t gr = row0 + row;
      const bool ok = gr < N && c < k;
      if (beta) lds[row * G::LDL + c] = ok ? dev::ld_d(P + gr * k + c) : 0.0;
      r[i] = ok ? dev::ld_d(R + gr * k + c) * dinv_at(dinv, gr) : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < G::RPT; ++i) {
      const int row = r0 + i * G::RS;
      const int64_t gr = row0 + row;
      double p = r[i];
      if (beta) p += dev::lds_row_dot<KP>(lds, row, bcol);
      if (gr < N && c < k) P[gr * k + c] = (T)p;
    }
    __syncthreads();
  }
}

// Y = c0 Y + c1 X C
template <typename T, int KP>
__global__ __launch_bounds__(256) void rmul_kernel(int64_t N, int k, const T* __restrict__ X, int ldx,
                                                   const double* __restrict__ C, double c0, double c1, T* Y, int ldy,
                                                   int64_t tps) {
  using G = TileGeom<KP>;
  __shared__ __align__(16) double lds[lds_doubles<KP>(1)];
  const int t = threadIdx.x, c = t % KP, r0 = t / KP;
  const int64_t slot = dev::xcd_slot(blockIdx.x, gridDim.x);
  const int64_t ntiles = (N + G::RT - 1) / G::RT;
  double ccol[KP];
  load_col<KP>(C, k, c, ccol);
  const int64_t tend = (slot + 1) * tps < ntiles ? (slot + 1) * tps : ntiles;
  for (int64_t tile = slot * tps; tile < tend; ++tile) {
    const int64_t row0 = tile * G::RT;
#pragma unroll
    for (int i = 0; i < G::RPT; ++i) {
      const int row = r0 + i * G::RS;
      const int64_t gr = row0 + row;
      lds[row * G::LDL + c] = (gr < N && c < k) ? dev::ld_d(X + gr * ldx + c) : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < G::RPT; ++i) {
      const int row = r0 + i * G::RS;
      const int64_t gr = row0 + row;
      if (gr < N && c < k) {
        double y = c1 * dev::lds_row_dot<KP>(lds, row, ccol);
        if (c0 != 0.0) y = fma(c0, dev::ld_d(Y + gr * ldy + c), y);
        Y[gr * ldy + c] = (T)y;
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------- casts / elementwise

// dst = coef * src * diag(s) (+ dst with accumulate), s inverted on request; with norm2 the scale of
// column c is sqrt(s[c]) (1 where s[c] is 0), so squared column norms scale without a host round trip.
template <typename S, typename D>
__global__ void cast_scale_kernel(int64_t N, int k, const S* src, int lds_, D* dst, int ldd, const double* s,
                                  int invert, int accumulate, int norm2, double coef) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N * k) return;
  const int64_t r = i / k;
  const int c = (int)(i % k);
  double v = (double)src[r * lds_ + c];
  if (s) {
    const double sc = norm2 ? (s[c] > 0.0 ? sqrt(s[c]) : 1.0) : s[c];
    v = invert ? v / sc : v * sc;
  }
  if (coef != 1.0) v = coef * v;
  if (accumulate) v += (double)dst[r * ldd + c];
  dst[r * ldd + c] = (D)v;
}

template <int KP>
void launch_gram_t(bkts_ctx ctx, int dtype, int64_t N, int k, const void* X, int ldx, const void* Y, int ldy,
                   double* G) {
  Slots s = make_slots<KP>(ctx, N);
  double* part = ctx->ws.get<double>("gram_partials", (size_t)KP * KP * s.nslots);
  ProfScope prof(ctx, BKTS_K_GRAM, 2.0 * N * k * esize(dtype));
  if (dtype == BKTS_F64)
    launch(ctx, (gram_kernel<double, KP>), dim3(s.nslots), dim3(256), 0, N, k,
                       static_cast<const double*>(X), ldx, static_cast<const double*>(Y), ldy, part, s.tps);
  else
    launch(ctx, (gram_kernel<float, KP>), dim3(s.nslots), dim3(256), 0, N, k,
                       static_cast<const float*>(X), ldx, static_cast<const float*>(Y), ldy, part, s.tps);
  BKTS_HIP(hipGetLastError());
  prof.end();
  finalize_gram(ctx, part, (int)s.nslots, k, KP, G);
  BKTS_HIP(hipGetLastError());
}

template <int KP>
void launch_colnorm_t(bkts_ctx ctx, int dtype, int64_t N, int k, const void* X, int ldx, double* out) {
  Slots s = make_slots<KP>(ctx, N);
  double* part = ctx->ws.get<double>("norm_partials", (size_t)KP * s.nslots);
  ProfScope prof(ctx, BKTS_K_NORMS, 1.0 * N * k * esize(dtype));
  if (dtype == BKTS_F64)
    launch(ctx, (colnorm_kernel<double, KP>), dim3(s.nslots), dim3(256), 0, N, k,
                       static_cast<const double*>(X), ldx, part, s.tps);
  else
    launch(ctx, (colnorm_kernel<float, KP>), dim3(s.nslots), dim3(256), 0, N, k,
                       static_cast<const float*>(X), ldx, part, s.tps);
  BKTS_HIP(hipGetLastError());
  prof.end();
  finalize_partials(ctx, part, (int)s.nslots, k, out);
  BKTS_HIP(hipGetLastError());
}

template <typename T, int KP, int NP>
void launch_coldots_vec(bkts_ctx ctx, int64_t N, int k, const DotPairs& d, double* const* out) {
  static_assert(KP * sizeof(T) >= 16, "rows of 16 bytes or more");
  int64_t nb = (int64_t)blocks_per_cu(reinterpret_cast<const void*>(coldots_vec_kernel<T, KP, NP>)) * ctx->num_cu;
  constexpr int64_t rows_per_step = 256 / (KP / (16 / (int)sizeof(T)));
  const int64_t steps = (N + rows_per_step - 1) / rows_per_step;
  if (nb > steps) nb = steps;
  if (nb < 1) nb = 1;
  double* part = ctx->ws.get<double>("dots_partials", (size_t)NP * KP * nb);
  ProfScope prof(ctx, BKTS_K_NORMS, 2.0 * NP * N * k * sizeof(T));
  launch(ctx, (coldots_vec_kernel<T, KP, NP>), dim3((unsigned)nb), dim3(256), 0, N, d, part);
  BKTS_HIP(hipGetLastError());
  prof.end();
  FoldSet sets[3];
  for (int p = 0; p < NP; ++p) sets[p] = FoldSet{part + (size_t)p * KP * nb, KP, 1, out[p]};
  finalize_sets(ctx, (int)nb, k, sets, NP);
}

template <int KP, int NP>
void launch_coldots_t(bkts_ctx ctx, int dtype, int64_t N, int k, const DotPairs& d, double* const* out) {
  auto al16 = [](const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; };
  bool vec = k == KP;
  for (int p = 0; p < NP; ++p) vec = vec && al16(d.x[p]) && al16(d.y[p]);
  if (vec && dtype == BKTS_F64) {
    if constexpr (KP >= 2) return launch_coldots_vec<double, KP, NP>(ctx, N, k, d, out);
  }
  if (vec && dtype == BKTS_F32) {
    if constexpr (KP >= 4) return launch_coldots_vec<float, KP, NP>(ctx, N, k, d, out);
  }
  Slots s = make_slots<KP>(ctx, N);
  double* part = ctx->ws.get<double>("dots_partials", (size_t)NP * KP * s.nslots);
  ProfScope prof(ctx, BKTS_K_NORMS, 2.0 * NP * N * k * esize(dtype));
  if (dtype == BKTS_F64)
    launch(ctx, (coldots_kernel<double, KP, NP>), dim3(s.nslots), dim3(256), 0, N, k, d, part, s.tps);
  else
    launch(ctx, (coldots_kernel<float, KP, NP>), dim3(s.nslots), dim3(256), 0, N, k, d, part, s.tps);
  BKTS_HIP(hipGetLastError());
  prof.end();
  FoldSet sets[3];
  for (int p = 0; p < NP; ++p) sets[p] = FoldSet{part + (size_t)p * KP * s.nslots, KP, 1, out[p]};
  finalize_sets(ctx, (int)s.nslots, k, sets, NP);
}

template <typename T, int KP>
void launch_cg_update_t(bkts_ctx ctx, int64_t N, int k, void* X, const void* P, void* R, const void* Q,
                        const double* alpha, const double* dinv,
                        double* gamma, double* Tm, double* nrm) {
  Slots s = make_slots<KP>(ctx, N);
  const size_t np = (size_t)KP * KP * s.nslots;
  double* pg = ctx->ws.get<double>("cg_pg", np);
  double* pt = ctx->ws.get<double>("cg_pt", np);
  double* pn = ctx->ws.get<double>("cg_pn", (size_t)KP * s.nslots);
  ProfScope prof(ctx, BKTS_K_CG_UPDATE, 6.0 * N * k * sizeof(T) + (dinv ? 8.0 * N : 0.0));
  launch(ctx, (cg_update_kernel<T, KP>), dim3(s.nslots), dim3(256), 0, N, k, static_cast<T*>(X),
                     static_cast<const T*>(P), static_cast<T*>(R), static_cast<const T*>(Q), alpha, dinv, pg, pt, pn, s.tps);
  BKTS_HIP(hipGetLastError());
  prof.end();
  finalize_gram(ctx, pg, (int)s.nslots, k, KP, gamma);
  finalize_gram(ctx, pt, (int)s.nslots, k, KP, Tm);
  finalize_partials(ctx, pn, (int)s.nslots, k, nrm);
  BKTS_HIP(hipGetLastError());
}

template <typename T, int KP>
void launch_cg_pupdate_t(bkts_ctx ctx, int64_t N, int k, void* P, const void* R, const double* beta,
                         const double* dinv) {
  Slots s = make_slots<KP>(ctx, N);
  ProfScope prof(ctx, BKTS_K_CG_PUPDATE, (beta ? 3.0 : 2.0) * N * k * sizeof(T) + (dinv ? 8.0 * N : 0.0));
  launch(ctx, (cg_pupdate_kernel<T, KP>), dim3(s.nslots), dim3(256), 0, N, k, static_cast<T*>(P),
                     static_cast<const T*>(R), beta, dinv, s.tps);
  BKTS_HIP(hipGetLastError());
}

template <typename T, int KP>
void launch_rmul_t(bkts_ctx ctx, int64_t N, int k, const void* X, int ldx, const double* C, double c0, double c1,
                   void* Y, int ldy) {
  Slots s = make_slots<KP>(ctx, N);
  ProfScope prof(ctx, BKTS_K_OTHER, (c0 != 0.0 ? 3.0 : 2.0) * N * k * sizeof(T));
  launch(ctx, (rmul_kernel<T, KP>), dim3(s.nslots), dim3(256), 0, N, k, static_cast<const T*>(X),
                     ldx, C, c0, c1, static_cast<T*>(Y), ldy, s.tps);
  BKTS_HIP(hipGetLastError());
}

#define BKTS_KP_DISPATCH(k, CALL)                                    \
  do {                                                               \
    if ((k) <= 1) { constexpr int KP = 1; CALL; }                    \
    else if ((k) <= 2) { constexpr int KP = 2; CALL; }               \
    else if ((k) <= 4) { constexpr int KP = 4; CALL; }               \
    else if ((k) <= 8) { constexpr int KP = 8; CALL; }               \
    else if ((k) <= 16) { constexpr int KP = 16; CALL; }             \
    else if ((k) <= 32) { constexpr int KP = 32; CALL; }             \
    else throw Error{BKTS_EINVAL, fmt("k=%d exceeds BKTS_MAX_K", (int)(k))}; \
  } while (0)

}  // namespace

void finalize_partials(bkts_ctx ctx, const double* partials, int nblocks, int nentries, double* out) {
  ProfScope prof(ctx, BKTS_K_SMALL, 8.0 * nblocks * nentries);
  launch(ctx, finalize_kernel, dim3(nentries), dim3(256), 0, partials, (int64_t)nblocks, 1, 1, 1,
                     out);
  BKTS_HIP(hipGetLastError());
}

void finalize_gram(bkts_ctx ctx, const double* partials, int nblocks, int k, int KP, double* out) {
  ProfScope prof(ctx, BKTS_K_SMALL, 8.0 * nblocks * k * k);
  launch(ctx, finalize_kernel, dim3(k * k), dim3(256), 0, partials, (int64_t)nblocks, k, KP, 0,
                     out);
  BKTS_HIP(hipGetLastError());
}

void finalize_sets(bkts_ctx ctx, int nblocks, int k, const FoldSet* sets, int nsets) {
  FoldArgs a{};
  a.nsets = nsets;
  a.k = k;
  a.nslots = nblocks;
  int total = 0;
  for (int i = 0; i < nsets; ++i) {
    a.set[i] = sets[i];
    total += sets[i].vector ? k : k * k;
  }
  ProfScope prof(ctx, BKTS_K_SMALL, 8.0 * nblocks * total);
  launch(ctx, finalize_sets_kernel, dim3(total), dim3(256), 0, a);
  BKTS_HIP(hipGetLastError());
}

void gram(bkts_ctx ctx, int dtype, int64_t N, int k, const void* X, int ldx, const void* Y, int ldy, double* G) {
  if (mf_eligible(k)) return mf_gram(ctx, dtype, N, k, X, ldx, Y, ldy, G);
  auto al16 = [](const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; };
  if (rk_eligible(k) && ldx == k && ldy == k && al16(X) && al16(Y)) return rk_gram(ctx, dtype, N, k, X, Y, G);
  BKTS_KP_DISPATCH(k, (launch_gram_t<KP>(ctx, dtype, N, k, X, ldx, Y, ldy, G)));
}

// ---------------------------------------------------------------- allocation-free Gram
// bkts_gram_noalloc keeps its per-workgroup partials in this fixed array instead of the context's
// workspace.  Each GPU holds its own copy until the process ends; host code never passes the array's
// name to a kernel (on the host it is only a stand-in) but the address hipGetSymbolAddress returned
// for the device, recorded once per device when a context is created on it.  Every workgroup writes
// all of its partials before the fold reads them, so nothing needs clearing between calls; calls
// that overlap on one GPU share the array and race.
constexpr size_t kScratchDoubles = 512 * 1024;  // 4 MiB
static __device__ __align__(256) double scratch[kScratchDoubles];

namespace {
std::mutex g_scratch_mu;
std::map<int, double*> g_scratch_addr;  // device ordinal -> that device's copy of `scratch`

double* scratch_of(int device) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_addr.find(device);
  BKTS_REQUIRE(it != g_scratch_addr.end(), "no scratch address recorded for device %d", device);
  return it->second;
}

template <int KP>
void gram_noalloc_t(bkts_ctx ctx, int dtype, int64_t N, int k, const void* X, int ldx, const void* Y, int ldy,
                    double* G) {
  double* part = scratch_of(ctx->device);
  Slots s = make_slots<KP>(ctx, N);
  const int64_t cap = (int64_t)(kScratchDoubles / (KP * KP));  // slots whose partials fit the array
  if (s.nslots > cap) {
    s.tps = (s.ntiles + cap - 1) / cap;
    s.nslots = (s.ntiles + s.tps - 1) / s.tps;
  }
  BKTS_REQUIRE((size_t)KP * KP * s.nslots <= kScratchDoubles,
               "bkts_gram_noalloc: %lld partials exceed the %zu-entry scratch array",
               (long long)(KP * KP * s.nslots), kScratchDoubles);
  if (dtype == BKTS_F64)
    launch(ctx, (gram_kernel<double, KP>), dim3(s.nslots), dim3(256), 0, N, k, static_cast<const double*>(X), ldx,
           static_cast<const double*>(Y), ldy, part, s.tps);
  else
    launch(ctx, (gram_kernel<float, KP>), dim3(s.nslots), dim3(256), 0, N, k, static_cast<const float*>(X), ldx,
           static_cast<const float*>(Y), ldy, part, s.tps);
  BKTS_HIP(hipGetLastError());
  launch(ctx, finalize_kernel, dim3(k * k), dim3(256), 0, (const double*)part, s.nslots, k, KP, 0, G);
  BKTS_HIP(hipGetLastError());
}
}  // namespace

void scratch_init(int device) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_addr.count(device)) return;
  void* p = nullptr;
  BKTS_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
  BKTS_REQUIRE(p, "hipGetSymbolAddress returned no address for the scratch array on device %d", device);
  g_scratch_addr[device] = static_cast<double*>(p);
}

void gram_noalloc(bkts_ctx ctx, int dtype, int64_t N, int k, const void* X, int ldx, const void* Y, int ldy,
                  double* G) {
  BKTS_KP_DISPATCH(k, (gram_noalloc_t<KP>(ctx, dtype, N, k, X, ldx, Y, ldy, G)));
}

void col_dots(bkts_ctx ctx, int dtype, int64_t N, int k, int npairs, const void* const* X, const void* const* Y,
              double* const* out) {
  BKTS_REQUIRE(npairs >= 1 && npairs <= 3, "col_dots: 1..3 pairs");
  DotPairs d{};
  for (int p = 0; p < npairs; ++p) {
    d.x[p] = X[p];
    d.y[p] = Y[p];
  }
  if (npairs == 1) BKTS_KP_DISPATCH(k, (launch_coldots_t<KP, 1>(ctx, dtype, N, k, d, out)));
  else if (npairs == 2) BKTS_KP_DISPATCH(k, (launch_coldots_t<KP, 2>(ctx, dtype, N, k, d, out)));
  else BKTS_KP_DISPATCH(k, (launch_coldots_t<KP, 3>(ctx, dtype, N, k, d, out)));
}

void colnorms2(bkts_ctx ctx, int dtype, int64_t N, int k, const void* X, int ldx, double* out) {
  // a full-width contiguous block of 16-byte rows: the vectorized column-dot pass of X with itself
  if (ldx == k && (reinterpret_cast<uintptr_t>(X) & 15) == 0 && (k & (k - 1)) == 0 &&
      k * (int)esize(dtype) >= 16) {
    const void* xs[1] = {X};
    double* os[1] = {out};
    return col_dots(ctx, dtype, N, k, 1, xs, xs, os);
  }
  BKTS_KP_DISPATCH(k, (launch_colnorm_t<KP>(ctx, dtype, N, k, X, ldx, out)));
}

void cg_update(bkts_ctx ctx, int dtype, int64_t N, int k, void* X, const void* P, void* R, const void* Q,
               const double* alpha, const double* dinv, double* gamma,
               double* Tm, double* nrm) {
  if (wide_eligible(dtype, k))
    return w_cg_update(ctx, N, k, static_cast<float*>(X), static_cast<const float*>(P), static_cast<float*>(R),
                       static_cast<const float*>(Q), alpha, dinv, gamma, Tm, nrm);
  if (mf_eligible(k)) return mf_cg_update(ctx, dtype, N, k, X, P, R, Q, alpha, dinv, gamma,
                                          Tm, nrm);
  if (rk_eligible(k)) return rk_cg_update(ctx, dtype, N, k, X, P, R, Q, alpha, dinv, gamma, Tm, nrm);
  if (dtype == BKTS_F64)
    BKTS_KP_DISPATCH(k, (launch_cg_update_t<double, KP>(ctx, N, k, X, P, R, Q, alpha, dinv,
                                                        gamma, Tm, nrm)));
  else
    BKTS_KP_DISPATCH(k, (launch_cg_update_t<float, KP>(ctx, N, k, X, P, R, Q, alpha, dinv,
                                                       gamma, Tm, nrm)));
}

void cg_pupdate(bkts_ctx ctx, int dtype, int64_t N, int k, void* P, const void* R, const double* beta,
                const double* dinv) {
  if (wide_eligible(dtype, k))
    return w_cg_pupdate(ctx, N, k, static_cast<float*>(P), static_cast<const float*>(R), beta, dinv);
  if (mf_eligible(k)) return mf_cg_pupdate(ctx, dtype, N, k, P, R, beta, dinv);
  if (rk_eligible(k)) return rk_cg_pupdate(ctx, dtype, N, k, P, R, beta, dinv);
  if (dtype == BKTS_F64)
    BKTS_KP_DISPATCH(k, (launch_cg_pupdate_t<double, KP>(ctx, N, k, P, R, beta, dinv)));
  else
    BKTS_KP_DISPATCH(k, (launch_cg_pupdate_t<float, KP>(ctx, N, k, P, R, beta, dinv)));
}

void block_rmul(bkts_ctx ctx, int dtype, int64_t N, int k, const void* X, int ldx, const double* C, double c0,
                double c1, void* Y, int ldy) {
  if (mf_eligible(k) && ldx == k && ldy == k) return mf_rmul(ctx, dtype, N, k, X, C, c0, c1, Y);
  if (rk_eligible(k) && ldx == k && ldy == k) return rk_rmul(ctx, dtype, N, k, X, C, c0, c1, Y);
  if (dtype == BKTS_F64)
    BKTS_KP_DISPATCH(k, (launch_rmul_t<double, KP>(ctx, N, k, X, ldx, C, c0, c1, Y, ldy)));
  else
    BKTS_KP_DISPATCH(k, (launch_rmul_t<float, KP>(ctx, N, k, X, ldx, C, c0, c1, Y, ldy)));
}

void block_cast_scale(bkts_ctx ctx, int64_t N, int k, int src_t, const void* src, int lds_, int dst_t, void* dst,
                      int ldd, const double* s, bool invert_s, bool accumulate, bool norm2, double coef) {
  const int64_t n = N * k;
  if (n == 0) return;
  dim3 g((n + 255) / 256), b(256);
  ProfScope prof(ctx, BKTS_K_CAST, (double)n * (esize(src_t) + esize(dst_t) * (accumulate ? 2 : 1)));
  if (lds_ == k && ldd == k && rk_cast(ctx, N, k, src_t, src, dst_t, dst, s, invert_s, accumulate, norm2, coef))
    return;
  const int iv = invert_s, ac = accumulate, n2 = norm2;
  if (src_t == BKTS_F64 && dst_t == BKTS_F32)
    launch(ctx, (cast_scale_kernel<double, float>), g, b, 0, N, k, static_cast<const double*>(src), lds_,
           static_cast<float*>(dst), ldd, s, iv, ac, n2, coef);
  else if (src_t == BKTS_F32 && dst_t == BKTS_F64)
    launch(ctx, (cast_scale_kernel<float, double>), g, b, 0, N, k, static_cast<const float*>(src), lds_,
           static_cast<double*>(dst), ldd, s, iv, ac, n2, coef);
  else if (src_t == BKTS_F64 && dst_t == BKTS_F64)
    launch(ctx, (cast_scale_kernel<double, double>), g, b, 0, N, k, static_cast<const double*>(src), lds_,
           static_cast<double*>(dst), ldd, s, iv, ac, n2, coef);
  else
    launch(ctx, (cast_scale_kernel<float, float>), g, b, 0, N, k, static_cast<const float*>(src), lds_,
           static_cast<float*>(dst), ldd, s, iv, ac, n2, coef);
  BKTS_HIP(hipGetLastError());
}

}  // namespace bkts

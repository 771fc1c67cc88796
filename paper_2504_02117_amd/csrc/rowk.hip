// Block-vector kernels for narrow blocks (k <= 4): one thread owns one whole row of every block.
// A row of k <= 4 values is one 4..32-byte vector load, the k x k right multiplications are
// register-only, and each thread keeps its share of the k x k Gram accumulators (FP64) in
// registers; consecutive threads own consecutive rows, so every access is coalesced and, for the
// sparse operator in SELL-C layout (C = 64), the matrix stream is contiguous per wave.
// Workgroups are persistent (sized to the resident capacity of the chip), each walks one
// contiguous XCD-aware row range, and leaves one partial per Gram entry (fixed-order folding).
#include "devcommon.hpp"
#include "internal.hpp"
#include "spd.hpp"

namespace bkts {
namespace {

template <typename T, int KP>
struct Row {
  T v[KP];
};

template <typename T, int KP>
__device__ __forceinline__ Row<T, KP> ld_row(const T* p, int k) {
  Row<T, KP> r;
  if constexpr (KP == 4 && sizeof(T) == 4) {
    const float4 q = *reinterpret_cast<const float4*>(p);
    r.v[0] = q.x; r.v[1] = q.y; r.v[2] = q.z; r.v[3] = q.w;
  } else if constexpr (KP == 4 && sizeof(T) == 8) {
    const double2 a = *reinterpret_cast<const double2*>(p);
    const double2 b = *reinterpret_cast<const double2*>(p + 2);
    r.v[0] = a.x; r.v[1] = a.y; r.v[2] = b.x; r.v[3] = b.y;
  } else if constexpr (KP == 2 && sizeof(T) == 8) {
    const double2 a = *reinterpret_cast<const double2*>(p);
    r.v[0] = a.x; r.v[1] = a.y;
  } else if constexpr (KP == 2 && sizeof(T) == 4) {
    const float2 a = *reinterpret_cast<const float2*>(p);
    r.v[0] = a.x; r.v[1] = a.y;
  } else {
#pragma unroll
    for (int j = 0; j < KP; ++j) r.v[j] = p[j];
  }
  (void)k;
  return r;
}

template <typename T, int KP>
__device__ __forceinline__ void st_row(T* p, const Row<T, KP>& r) {
  if constexpr (KP == 4 && sizeof(T) == 4) {
    *reinterpret_cast<float4*>(p) = float4{r.v[0], r.v[1], r.v[2], r.v[3]};
  } else if constexpr (KP == 4 && sizeof(T) == 8) {
    *reinterpret_cast<double2*>(p) = double2{r.v[0], r.v[1]};
    *reinterpret_cast<double2*>(p + 2) = double2{r.v[2], r.v[3]};
  } else if constexpr (KP == 2 && sizeof(T) == 8) {
    *reinterpret_cast<double2*>(p) = double2{r.v[0], r.v[1]};
  } else if constexpr (KP == 2 && sizeof(T) == 4) {
    *reinterpret_cast<float2*>(p) = float2{r.v[0], r.v[1]};
  } else {
#pragma unroll
    for (int j = 0; j < KP; ++j) p[j] = r.v[j];
  }
}

struct RowRange {
  int64_t begin, end;
};

// Contiguous row range of this (XCD-remapped) workgroup, in whole 256-row chunks.
__device__ __forceinline__ RowRange block_rows(int64_t N) {
  const int64_t slot = dev::xcd_slot(blockIdx.x, gridDim.x);
  const int64_t chunks = (N + 255) / 256;
  const int64_t per = (chunks + gridDim.x - 1) / gridDim.x;
  RowRange r;
  r.begin = slot * per * 256;
  r.end = (slot + 1) * per * 256;
  if (r.begin > N) r.begin = N;
  if (r.end > N) r.end = N;
  return r;
}

// Fold acc[NA] (identical layout in every thread) over the workgroup in a fixed order and store
// partials[e * nslots + slot].  Ends with a barrier.
template <int NA>
__device__ void fold_block(double (&acc)[NA], double* red, double* partials) {
#pragma unroll
  for (int off = 1; off < 64; off <<= 1)
#pragma unroll
    for (int a = 0; a < NA; ++a) acc[a] += __shfl_xor(acc[a], off);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  if (l == 0) {
#pragma unroll
    for (int a = 0; a < NA; ++a) red[w * NA + a] = acc[a];
  }
  __syncthreads();
  const int64_t slot = dev::xcd_slot(blockIdx.x, gridDim.x);
  for (int e = threadIdx.x; e < NA; e += dev::kThreads)
    partials[(int64_t)e * gridDim.x + slot] = ((red[e] + red[NA + e]) + red[2 * NA + e]) + red[3 * NA + e];
  __syncthreads();
}

template <typename T>
struct RkSpmmArgs {
  int64_t N;
  int k;
  const int32_t* rowptr;
  const int32_t* col;
  const T* val;
  const int64_t* sptr;
  const int32_t* sw;
  int C;
  double alpha, beta;
  const T* P;
  T* Q;
  double* partials;  // G = P^T Q, entries a*KP + b
};

// Q = alpha P + beta K P (arithmetic in T) and G = P^T Q (FP64).
template <typename T, int KP, bool SELL>
__global__ __launch_bounds__(256) void rk_spmm_gram_kernel(RkSpmmArgs<T> a) {
  __shared__ double red[4 * KP * KP];
  double g[KP * KP];
#pragma unroll
  for (int e = 0; e < KP * KP; ++e) g[e] = 0.0;
  const RowRange rr = block_rows(a.N);
  for (int64_t r = rr.begin + threadIdx.x; r < rr.end; r += dev::kThreads) {
    int64_t base, stride, len;
    if constexpr (SELL) {
      const int64_t s = r / a.C;
      base = a.sptr[s] + (r - s * a.C);
      stride = a.C;
      len = a.sw[s];
    } else {
      base = a.rowptr[r];
      stride = 1;
      len = a.rowptr[r + 1] - base;
    }
    T acc[KP];
#pragma unroll
    for (int j = 0; j < KP; ++j) acc[j] = T(0);
    constexpr int U = 8;
    for (int64_t j0 = 0; j0 < len; j0 += U) {
      T v[U];
      int32_t ci[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const bool ok = j0 + u < len;
        const int64_t e = base + (j0 + u) * stride;
        v[u] = ok ? a.val[e] : T(0);
        ci[u] = ok ? a.col[e] : (int32_t)r;
      }
      Row<T, KP> x[U];
#pragma unroll
      for (int u = 0; u < U; ++u) x[u] = ld_row<T, KP>(a.P + (int64_t)ci[u] * KP, a.k);
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int j = 0; j < KP; ++j) acc[j] = fma(v[u], x[u].v[j], acc[j]);
    }
    const Row<T, KP> p = ld_row<T, KP>(a.P + r * KP, a.k);
    Row<T, KP> q;
#pragma unroll
    for (int j = 0; j < KP; ++j) q.v[j] = (T)a.beta * acc[j] + (T)a.alpha * p.v[j];
    st_row<T, KP>(a.Q + r * KP, q);
#pragma unroll
    for (int i = 0; i < KP; ++i)
#pragma unroll
      for (int j = 0; j < KP; ++j) g[i * KP + j] = fma((double)p.v[i], (double)q.v[j], g[i * KP + j]);
  }
  fold_block<KP * KP>(g, red, a.partials);
}

// Stencil form (symmetric 5/7-point operator on a structured grid): no column-index stream;
// coef holds d and the na off-diagonal arrays o_a (entry K[r, r + s_a]), each of length N.
template <typename T>
struct RkStArgs {
  int64_t N;
  int na;
  int64_t s[3];
  const T* coef;
  double alpha, beta;
  const T* P;
  T* Q;
  double* partials;
};

// G rows per thread per step (256 apart), all their loads issued before the first FMA: four for
// FP32 rows of four columns (100 VGPRs, 5% faster than two at 128^3; six or more rows cost occupancy
// and run 30% slower), two otherwise.
template <typename T, int KP>
__global__ __launch_bounds__(256) void rk_st_spmm_gram_kernel(RkStArgs<T> a) {
  constexpr int G = (sizeof(T) == 4 && KP == 4) ? 4 : 2;
  __shared__ double red[4 * KP * KP];
  double g[KP * KP];
#pragma unroll
  for (int e = 0; e < KP * KP; ++e) g[e] = 0.0;
  const int64_t N = a.N;
  // units of G chunks walked per XCD slab (the neighbour planes stay in the XCD's L2); every load of
  // a unit is issued before the arithmetic: rows past N read row N - 1, a neighbour past either end
  // reads the row itself, and both come with zero weights
  const dev::ChunkWalk walk = dev::xcd_chunks((N + G * dev::kThreads - 1) / (G * dev::kThreads));
  for (int64_t u = walk.first; u < walk.end; u += walk.step) {
    const int64_t r0 = u * (G * dev::kThreads) + threadIdx.x;
    int64_t r[G];
    bool ok[G];
    T dg[G], up[G][3], lo[G][3];
    Row<T, KP> p[G], xu[G][3], xl[G][3];
#pragma unroll
    for (int h = 0; h < G; ++h) {
      r[h] = r0 + h * dev::kThreads;
      ok[h] = r[h] < N;
      const int64_t rr = ok[h] ? r[h] : N - 1;
      dg[h] = __builtin_nontemporal_load(a.coef + rr) * T(ok[h] ? 1 : 0);
      p[h] = ld_row<T, KP>(a.P + rr * KP, KP);
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        const bool has = q < a.na;
        const int64_t s = has ? a.s[q] : 0;
        const bool uo = has && rr + s < N, lk = has && rr - s >= 0;
        const int64_t ru = uo ? rr + s : rr, rl = lk ? rr - s : rr;
        const T* oq = a.coef + (1 + (has ? q : 0)) * N;
        up[h][q] = oq[rr] * T(uo ? 1 : 0);
        lo[h][q] = oq[rl] * T(lk ? 1 : 0);
        xu[h][q] = ld_row<T, KP>(a.P + ru * KP, KP);
        xl[h][q] = ld_row<T, KP>(a.P + rl * KP, KP);
      }
    }
#pragma unroll
    for (int h = 0; h < G; ++h) {
      if (!ok[h]) continue;
      T acc[KP];
#pragma unroll
      for (int j = 0; j < KP; ++j) acc[j] = dg[h] * p[h].v[j];
#pragma unroll
      for (int q = 0; q < 3; ++q) {
#pragma unroll
        for (int j = 0; j < KP; ++j) acc[j] = fma(lo[h][q], xl[h][q].v[j], acc[j]);
#pragma unroll
        for (int j = 0; j < KP; ++j) acc[j] = fma(up[h][q], xu[h][q].v[j], acc[j]);
      }
      Row<T, KP> qv;
#pragma unroll
      for (int j = 0; j < KP; ++j) qv.v[j] = (T)a.beta * acc[j] + (T)a.alpha * p[h].v[j];
      st_row<T, KP>(a.Q + r[h] * KP, qv);
#pragma unroll
      for (int i = 0; i < KP; ++i)
#pragma unroll
        for (int j = 0; j < KP; ++j) g[i * KP + j] = fma((double)p[h].v[i], (double)qv.v[j], g[i * KP + j]);
    }
  }
  fold_block<KP * KP>(g, red, a.partials);
}

struct RkUpdArgs {
  int64_t N;
  void* X;
  const void* P;
  void* R;
  const void* Q;
  const double* alpha;
  const double* dinv;  // inverse Jacobi diagonal, or null for no preconditioning
  double* partials;  // [gamma (KP^2) | T (KP^2) | nrm (KP)] entries
};

// X += P alpha; R -= Q alpha; Z = D^-1 R; gamma = R^T Z; T = Q^T Z; nrm = diag(R^T R).  Two rows per
// thread per step, with the loads of both issued before the arithmetic.
template <typename T, int KP>
__global__ __launch_bounds__(256) void rk_cg_update_kernel(RkUpdArgs a) {
  constexpr int NA = 2 * KP * KP + KP;
  __shared__ double red[4 * NA];
  double al[KP * KP];
#pragma unroll
  for (int e = 0; e < KP * KP; ++e) al[e] = a.alpha[e];
  double acc[NA];
#pragma unroll
  for (int e = 0; e < NA; ++e) acc[e] = 0.0;
  const T* P = static_cast<const T*>(a.P);
  const T* Q = static_cast<const T*>(a.Q);
  T* X = static_cast<T*>(a.X);
  T* R = static_cast<T*>(a.R);
  const RowRange rr = block_rows(a.N);
  constexpr int GR = 2;  // rows per thread per step (256 apart), all loads issued first
  for (int64_t r0 = rr.begin + threadIdx.x; r0 < rr.end; r0 += GR * dev::kThreads) {
    Row<T, KP> p[GR], q[GR], x[GR], rv[GR];
    double dv[GR];
    bool ok[GR];
#pragma unroll
    for (int h = 0; h < GR; ++h) {
      const int64_t r = r0 + h * dev::kThreads;
      ok[h] = r < rr.end;
      if (ok[h]) {
        p[h] = ld_row<T, KP>(P + r * KP, KP);
        q[h] = ld_row<T, KP>(Q + r * KP, KP);
        x[h] = ld_row<T, KP>(X + r * KP, KP);
        rv[h] = ld_row<T, KP>(R + r * KP, KP);
      }
      dv[h] = (ok[h] && a.dinv) ? a.dinv[r] : 1.0;
    }
#pragma unroll
    for (int h = 0; h < GR; ++h) {
      if (!ok[h]) continue;
      const int64_t r = r0 + h * dev::kThreads;
      double z[KP], rn[KP];
#pragma unroll
      for (int c = 0; c < KP; ++c) {
        double xs = (double)x[h].v[c], rs = (double)rv[h].v[c];
#pragma unroll
        for (int j = 0; j < KP; ++j) {
          xs = fma((double)p[h].v[j], al[j * KP + c], xs);
          rs = fma(-(double)q[h].v[j], al[j * KP + c], rs);
        }
        x[h].v[c] = (T)xs;
        rv[h].v[c] = (T)rs;
        rn[c] = (double)rv[h].v[c];
        z[c] = rn[c] * dv[h];
      }
      st_row<T, KP>(X + r * KP, x[h]);
      st_row<T, KP>(R + r * KP, rv[h]);
#pragma unroll
      for (int i = 0; i < KP; ++i)
#pragma unroll
        for (int j = 0; j < KP; ++j) {
          acc[i * KP + j] = fma(rn[i], z[j], acc[i * KP + j]);
          acc[KP * KP + i * KP + j] = fma((double)q[h].v[i], z[j], acc[KP * KP + i * KP + j]);
        }
#pragma unroll
      for (int c = 0; c < KP; ++c) acc[2 * KP * KP + c] = fma(rn[c], rn[c], acc[2 * KP * KP + c]);
    }
  }
  fold_block<NA>(acc, red, a.partials);
}

// X += P alpha (MODE 0, 2) and R -= Q alpha (MODE 0, 1), and nothing else (the reductions that
// follow come from another pass).  Two rows per thread per step, loads of both issued first.
template <typename T, int KP, int MODE>
__global__ __launch_bounds__(256) void rk_cg_xr_kernel(int64_t N, T* __restrict__ X, const T* __restrict__ P,
                                                       T* __restrict__ R, const T* __restrict__ Q,
                                                       const double* alpha) {
  constexpr bool DX = MODE != 1, DR = MODE != 2;
  double al[KP * KP];
#pragma unroll
  for (int e = 0; e < KP * KP; ++e) al[e] = alpha[e];
  const RowRange rr = block_rows(N);
  constexpr int GR = 2;
  for (int64_t r0 = rr.begin + threadIdx.x; r0 < rr.end; r0 += GR * dev::kThreads) {
    Row<T, KP> p[GR], q[GR], x[GR], rv[GR];
    bool ok[GR];
#pragma unroll
    for (int h = 0; h < GR; ++h) {
      const int64_t r = r0 + h * dev::kThreads;
      ok[h] = r < rr.end;
      if (ok[h]) {
        if (DX) {
          p[h] = ld_row<T, KP>(P + r * KP, KP);
          x[h] = ld_row<T, KP>(X + r * KP, KP);
        }
        if (DR) {
          q[h] = ld_row<T, KP>(Q + r * KP, KP);
          rv[h] = ld_row<T, KP>(R + r * KP, KP);
        }
      }
    }
#pragma unroll
    for (int h = 0; h < GR; ++h) {
      if (!ok[h]) continue;
      const int64_t r = r0 + h * dev::kThreads;
#pragma unroll
      for (int c = 0; c < KP; ++c) {
        if (DX) {
          double xs = (double)x[h].v[c];
#pragma unroll
          for (int j = 0; j < KP; ++j) xs = fma((double)p[h].v[j], al[j * KP + c], xs);
          x[h].v[c] = (T)xs;
        }
        if (DR) {
          double rs = (double)rv[h].v[c];
#pragma unroll
          for (int j = 0; j < KP; ++j) rs = fma(-(double)q[h].v[j], al[j * KP + c], rs);
          rv[h].v[c] = (T)rs;
        }
      }
      if (DX) st_row<T, KP>(X + r * KP, x[h]);
      if (DR) st_row<T, KP>(R + r * KP, rv[h]);
    }
  }
}

// X += P alpha and P = Z + P beta from the same read of the old P (one row per thread per step).
template <typename T, int KP>
__global__ __launch_bounds__(256) void rk_cg_xp_kernel(int64_t N, T* __restrict__ X, T* __restrict__ P,
                                                       const T* __restrict__ Z, const double* alpha,
                                                       const double* beta, int x_init) {
  double al[KP * KP], be[KP * KP];
#pragma unroll
  for (int e = 0; e < KP * KP; ++e) {
    al[e] = alpha[e];
    be[e] = beta[e];
  }
  const RowRange rr = block_rows(N);
  for (int64_t r = rr.begin + threadIdx.x; r < rr.end; r += dev::kThreads) {
    const Row<T, KP> p = ld_row<T, KP>(P + r * KP, KP);
    Row<T, KP> x;
    if (x_init) {  // the first update of a solve from zero: X = P alpha, X not read
#pragma unroll
      for (int c = 0; c < KP; ++c) x.v[c] = T(0);
    } else {
      x = ld_row<T, KP>(X + r * KP, KP);
    }
    Row<T, KP> z = ld_row<T, KP>(Z + r * KP, KP);
#pragma unroll
    for (int c = 0; c < KP; ++c) {
      double xs = (double)x.v[c], ps = (double)z.v[c];
#pragma unroll
      for (int j = 0; j < KP; ++j) {
        xs = fma((double)p.v[j], al[j * KP + c], xs);
        ps = fma((double)p.v[j], be[j * KP + c], ps);
      }
      x.v[c] = (T)xs;
      z.v[c] = (T)ps;
    }
    st_row<T, KP>(X + r * KP, x);
    st_row<T, KP>(P + r * KP, z);
  }
}

// P = D^-1 R + P beta   (beta == nullptr: P = D^-1 R)
template <typename T, int KP>
__global__ __launch_bounds__(256) void rk_cg_pupdate_kernel(int64_t N, T* __restrict__ P, const T* __restrict__ R,
                                                            const double* beta, const double* dinv) {
  double be[KP * KP];
#pragma unroll
  for (int e = 0; e < KP * KP; ++e) be[e] = beta ? beta[e] : 0.0;
  const RowRange rr = block_rows(N);
  for (int64_t r = rr.begin + threadIdx.x; r < rr.end; r += dev::kThreads) {
    const Row<T, KP> rv = ld_row<T, KP>(R + r * KP, KP);
    const double dv = dinv ? dinv[r] : 1.0;
    Row<T, KP> out;
    if (beta) {
      const Row<T, KP> p = ld_row<T, KP>(P + r * KP, KP);
#pragma unroll
      for (int c = 0; c < KP; ++c) {
        double s = (double)rv.v[c] * dv;
#pragma unroll
        for (int j = 0; j < KP; ++j) s = fma((double)p.v[j], be[j * KP + c], s);
        out.v[c] = (T)s;
      }
    } else {
#pragma unroll
      for (int c = 0; c < KP; ++c) out.v[c] = (T)((double)rv.v[c] * dv);
    }
    st_row<T, KP>(P + r * KP, out);
  }
}

// G = X^T Y (contiguous blocks)
template <typename T, int KP>
__global__ __launch_bounds__(256) void rk_gram_kernel(int64_t N, const T* __restrict__ X, const T* __restrict__ Y,
                                                      double* partials) {
  __shared__ double red[4 * KP * KP];
  double g[KP * KP];
#pragma unroll
  for (int e = 0; e < KP * KP; ++e) g[e] = 0.0;
  const RowRange rr = block_rows(N);
  for (int64_t r = rr.begin + threadIdx.x; r < rr.end; r += dev::kThreads) {
    const Row<T, KP> x = ld_row<T, KP>(X + r * KP, KP);
    const Row<T, KP> y = ld_row<T, KP>(Y + r * KP, KP);
#pragma unroll
    for (int i = 0; i < KP; ++i)
#pragma unroll
      for (int j = 0; j < KP; ++j) g[i * KP + j] = fma((double)x.v[i], (double)y.v[j], g[i * KP + j]);
  }
  fold_block<KP * KP>(g, red, partials);
}

// G1 = X1^T Y and G2 = X2^T Y in one pass over the three blocks (two rows per thread per step)
template <typename T, int KP>
__global__ __launch_bounds__(256) void rk_gram2_kernel(int64_t N, const T* __restrict__ X1, const T* __restrict__ X2,
                                                       const T* __restrict__ Y, double* partials) {
  constexpr int NA = 2 * KP * KP;
  constexpr int GR = 2;
  __shared__ double red[4 * NA];
  double g[NA];
#pragma unroll
  for (int e = 0; e < NA; ++e) g[e] = 0.0;
  const RowRange rr = block_rows(N);
  for (int64_t r0 = rr.begin + threadIdx.x; r0 < rr.end; r0 += GR * dev::kThreads) {
    Row<T, KP> a[GR], b[GR], y[GR];
    bool ok[GR];
#pragma unroll
    for (int h = 0; h < GR; ++h) {
      const int64_t r = r0 + h * dev::kThreads;
      ok[h] = r < rr.end;
      if (ok[h]) {
        a[h] = ld_row<T, KP>(X1 + r * KP, KP);
        b[h] = ld_row<T, KP>(X2 + r * KP, KP);
        y[h] = ld_row<T, KP>(Y + r * KP, KP);
      }
    }
#pragma unroll
    for (int h = 0; h < GR; ++h) {
      if (!ok[h]) continue;
#pragma unroll
      for (int i = 0; i < KP; ++i)
#pragma unroll
        for (int j = 0; j < KP; ++j) {
          g[i * KP + j] = fma((double)a[h].v[i], (double)y[h].v[j], g[i * KP + j]);
          g[KP * KP + i * KP + j] = fma((double)b[h].v[i], (double)y[h].v[j], g[KP * KP + i * KP + j]);
        }
    }
  }
  fold_block<NA>(g, red, partials);
}

// Y = c0 Y + c1 X C (contiguous blocks)
template <typename T, int KP>
__global__ __launch_bounds__(256) void rk_rmul_kernel(int64_t N, const T* __restrict__ X, const double* Cm, double c0,
                                                      double c1, T* Y) {
  double cm[KP * KP];
#pragma unroll
  for (int e = 0; e < KP * KP; ++e) cm[e] = c1 * Cm[e];
  const RowRange rr = block_rows(N);
  for (int64_t r = rr.begin + threadIdx.x; r < rr.end; r += dev::kThreads) {
    const Row<T, KP> x = ld_row<T, KP>(X + r * KP, KP);
    Row<T, KP> y;
    if (c0 != 0.0) y = ld_row<T, KP>(Y + r * KP, KP);
#pragma unroll
    for (int c = 0; c < KP; ++c) {
      double s = c0 != 0.0 ? c0 * (double)y.v[c] : 0.0;
#pragma unroll
      for (int j = 0; j < KP; ++j) s = fma((double)x.v[j], cm[j * KP + c], s);
      y.v[c] = (T)s;
    }
    st_row<T, KP>(Y + r * KP, y);
  }
}

// Persistent grid: the resident capacity of the chip for this kernel (occupancy x CUs), capped by
// the number of 256-row chunks.
template <typename K>
int64_t rk_grid(bkts_ctx ctx, K kernel, int64_t N) {
  int64_t nb = (int64_t)blocks_per_cu(reinterpret_cast<const void*>(kernel)) * ctx->num_cu;
  const int64_t chunks = (N + 255) / 256;
  if (nb > chunks) nb = chunks;
  if (nb >= dev::kXcd) nb -= nb % dev::kXcd;  // whole rounds over the XCDs
  return nb < 1 ? 1 : nb;
}

// dst = coef * src * diag(s) (+ dst with accumulate) for contiguous rows of KP <= 4 columns, one row
// per thread with vector loads; the column scales as in block_cast_scale (s inverted on request, or
// the square roots of squared norms, 1 for a zero column).
template <typename S, typename D, int KP>
__global__ __launch_bounds__(256) void rk_cast_kernel(int64_t N, const S* __restrict__ src, D* dst, const double* s,
                                                      int invert, int accumulate, int norm2, double coef) {
  const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (r >= N) return;
  double sc[KP];
#pragma unroll
  for (int c = 0; c < KP; ++c) sc[c] = s ? (norm2 ? (s[c] > 0.0 ? sqrt(s[c]) : 1.0) : s[c]) : 1.0;
  const Row<S, KP> x = ld_row<S, KP>(src + r * KP, KP);
  Row<D, KP> y;
  if (accumulate) y = ld_row<D, KP>(dst + r * KP, KP);
#pragma unroll
  for (int c = 0; c < KP; ++c) {
    double v = (double)x.v[c];
    if (s) v = invert ? v / sc[c] : v * sc[c];
    if (coef != 1.0) v = coef * v;
    if (accumulate) v += (double)y.v[c];
    y.v[c] = (D)v;
  }
  st_row<D, KP>(dst + r * KP, y);
}

}  // namespace

bool rk_eligible(int k) { return k == 1 || k == 2 || k == 4; }

#define BKTS_RK_DISPATCH(k, CALL)                 \
  do {                                            \
    if ((k) == 1) { constexpr int KP = 1; CALL; } \
    else if ((k) == 2) { constexpr int KP = 2; CALL; } \
    else { constexpr int KP = 4; CALL; }          \
  } while (0)

template <typename T, int KP>
static void rk_st_spmm_gram_t(bkts_ctx ctx, const bkts_op_s& op, double alpha, const void* P, double beta, void* Q,
                              double* G, const CgTail* tail) {
  RkStArgs<T> a{};
  a.N = op.N;
  a.na = op.st_na;
  for (int q = 0; q < 3; ++q) a.s[q] = op.st_off[q];
  if constexpr (sizeof(T) == 8)
    a.coef = op.st_coef.as<double>();
  else
    a.coef = op.st_coef32.as<float>();
  a.alpha = alpha;
  a.beta = beta;
  a.P = static_cast<const T*>(P);
  a.Q = static_cast<T*>(Q);
  const double sv = sizeof(T);
  ProfScope prof(ctx, BKTS_K_SPMM, (1.0 + op.st_na) * op.N * sv + 2.0 * op.N * KP * sv);
  const int64_t nb = rk_grid(ctx, rk_st_spmm_gram_kernel<T, KP>, op.N);
  a.partials = ctx->ws.get<double>("rk_sg_part", (size_t)KP * KP * nb);
  launch(ctx, (rk_st_spmm_gram_kernel<T, KP>), dim3(nb), dim3(256), 0, a);
  BKTS_HIP(hipGetLastError());
  prof.end();
  if (!tail) return finalize_gram(ctx, a.partials, (int)nb, KP, KP, G);
  fold_solve(ctx, 0, KP, KP, a.partials, nb, *tail);
}

template <typename T, int KP>
static void rk_spmm_gram_t(bkts_ctx ctx, const bkts_op_s& op, double alpha, const void* P, double beta, void* Q,
                           double* G, const CgTail* tail) {
  if (op.st_na > 0) return rk_st_spmm_gram_t<T, KP>(ctx, op, alpha, P, beta, Q, G, tail);
  const bool sell = op.format == BKTS_FMT_SELL;
  RkSpmmArgs<T> a{};
  a.N = op.N;
  a.k = KP;
  a.rowptr = op.rowptr.as<int32_t>();
  a.col = sell ? op.sell_col.as<int32_t>() : op.col.as<int32_t>();
  if constexpr (sizeof(T) == 8)
    a.val = sell ? op.sell_val.as<double>() : op.val.as<double>();
  else
    a.val = sell ? op.sell_val32.as<float>() : op.val32.as<float>();
  a.sptr = op.sell_ptr.as<int64_t>();
  a.sw = op.sell_w.as<int32_t>();
  a.C = op.sell_C;
  a.alpha = alpha;
  a.beta = beta;
  a.P = static_cast<const T*>(P);
  a.Q = static_cast<T*>(Q);
  const double sv = sizeof(T);
  ProfScope prof(ctx, BKTS_K_SPMM, op.nnz * (sv + 4.0) + 4.0 * (op.N + 1) + 2.0 * op.N * KP * sv);
  int64_t nb;
  if (sell) {
    nb = rk_grid(ctx, rk_spmm_gram_kernel<T, KP, true>, op.N);
    a.partials = ctx->ws.get<double>("rk_sg_part", (size_t)KP * KP * nb);
    launch(ctx, (rk_spmm_gram_kernel<T, KP, true>), dim3(nb), dim3(256), 0, a);
  } else {
    nb = rk_grid(ctx, rk_spmm_gram_kernel<T, KP, false>, op.N);
    a.partials = ctx->ws.get<double>("rk_sg_part", (size_t)KP * KP * nb);
    launch(ctx, (rk_spmm_gram_kernel<T, KP, false>), dim3(nb), dim3(256), 0, a);
  }
  BKTS_HIP(hipGetLastError());
  prof.end();
  if (!tail) return finalize_gram(ctx, a.partials, (int)nb, KP, KP, G);
  fold_solve(ctx, 0, KP, KP, a.partials, nb, *tail);
}

void rk_spmm_gram(bkts_ctx ctx, const bkts_op_s& op, int dtype, int k, double alpha, const void* P, double beta,
                  void* Q, double* G, const CgTail* tail) {
  if (dtype == BKTS_F64)
    BKTS_RK_DISPATCH(k, (rk_spmm_gram_t<double, KP>(ctx, op, alpha, P, beta, Q, G, tail)));
  else
    BKTS_RK_DISPATCH(k, (rk_spmm_gram_t<float, KP>(ctx, op, alpha, P, beta, Q, G, tail)));
}

template <typename T, int KP>
static void rk_cg_update_t(bkts_ctx ctx, int64_t N, void* X, const void* P, void* R, const void* Q,
                           const double* alpha, const double* dinv,
                           double* gamma, double* Tm, double* nrm, const CgTail* tail) {
  constexpr int NA = 2 * KP * KP + KP;
  const int64_t nb = rk_grid(ctx, rk_cg_update_kernel<T, KP>, N);
  double* part = ctx->ws.get<double>("rk_upd_part", (size_t)NA * nb);
  RkUpdArgs a{N, X, P, R, Q, alpha, dinv, part};
  ProfScope prof(ctx, BKTS_K_CG_UPDATE, 6.0 * N * KP * sizeof(T) + (dinv ? 8.0 * N : 0.0));
  launch(ctx, (rk_cg_update_kernel<T, KP>), dim3(nb), dim3(256), 0, a);
  BKTS_HIP(hipGetLastError());
  prof.end();
  if (tail) {
    fold_solve(ctx, 1, KP, KP, part, nb, *tail);
    return;
  }
  const FoldSet sets[3] = {{part, KP, 0, gamma}, {part + (size_t)KP * KP * nb, KP, 0, Tm},
                           {part + (size_t)2 * KP * KP * nb, KP, 1, nrm}};
  finalize_sets(ctx, (int)nb, KP, sets, 3);
}

void rk_cg_update(bkts_ctx ctx, int dtype, int64_t N, int k, void* X, const void* P, void* R, const void* Q,
                  const double* alpha, const double* dinv, double* gamma, double* Tm, double* nrm,
                  const CgTail* tail) {
  if (dtype == BKTS_F64)
    BKTS_RK_DISPATCH(k, (rk_cg_update_t<double, KP>(ctx, N, X, P, R, Q, alpha, dinv, gamma, Tm, nrm, tail)));
  else
    BKTS_RK_DISPATCH(k, (rk_cg_update_t<float, KP>(ctx, N, X, P, R, Q, alpha, dinv, gamma, Tm, nrm, tail)));
}

template <typename T, int KP, int MODE>
static void rk_cg_xr_t(bkts_ctx ctx, int64_t N, void* X, const void* P, void* R, const void* Q, const double* alpha) {
  const int64_t nb = rk_grid(ctx, rk_cg_xr_kernel<T, KP, MODE>, N);
  ProfScope prof(ctx, BKTS_K_CG_UPDATE, (MODE == 0 ? 6.0 : 3.0) * N * KP * sizeof(T));
  launch(ctx, (rk_cg_xr_kernel<T, KP, MODE>), dim3(nb), dim3(256), 0, N, static_cast<T*>(X),
         static_cast<const T*>(P), static_cast<T*>(R), static_cast<const T*>(Q), alpha);
  BKTS_HIP(hipGetLastError());
}

void rk_cg_xr_update(bkts_ctx ctx, int dtype, int64_t N, int k, void* X, const void* P, void* R, const void* Q,
                     const double* alpha) {
  if (dtype == BKTS_F64)
    BKTS_RK_DISPATCH(k, (rk_cg_xr_t<double, KP, 0>(ctx, N, X, P, R, Q, alpha)));
  else
    BKTS_RK_DISPATCH(k, (rk_cg_xr_t<float, KP, 0>(ctx, N, X, P, R, Q, alpha)));
}

void rk_cg_r_update(bkts_ctx ctx, int dtype, int64_t N, int k, void* R, const void* Q, const double* alpha) {
  if (dtype == BKTS_F64)
    BKTS_RK_DISPATCH(k, (rk_cg_xr_t<double, KP, 1>(ctx, N, nullptr, nullptr, R, Q, alpha)));
  else
    BKTS_RK_DISPATCH(k, (rk_cg_xr_t<float, KP, 1>(ctx, N, nullptr, nullptr, R, Q, alpha)));
}

void rk_cg_x_update(bkts_ctx ctx, int dtype, int64_t N, int k, void* X, const void* P, const double* alpha) {
  if (dtype == BKTS_F64)
    BKTS_RK_DISPATCH(k, (rk_cg_xr_t<double, KP, 2>(ctx, N, X, P, nullptr, nullptr, alpha)));
  else
    BKTS_RK_DISPATCH(k, (rk_cg_xr_t<float, KP, 2>(ctx, N, X, P, nullptr, nullptr, alpha)));
}

template <typename T, int KP>
static void rk_cg_xp_t(bkts_ctx ctx, int64_t N, void* X, void* P, const void* Z, const double* alpha,
                       const double* beta, bool x_init) {
  const int64_t nb = rk_grid(ctx, rk_cg_xp_kernel<T, KP>, N);
  ProfScope prof(ctx, BKTS_K_CG_PUPDATE, (x_init ? 4.0 : 5.0) * N * KP * sizeof(T));
  launch(ctx, (rk_cg_xp_kernel<T, KP>), dim3(nb), dim3(256), 0, N, static_cast<T*>(X), static_cast<T*>(P),
         static_cast<const T*>(Z), alpha, beta, x_init ? 1 : 0);
  BKTS_HIP(hipGetLastError());
}

void rk_cg_xp_update(bkts_ctx ctx, int dtype, int64_t N, int k, void* X, void* P, const void* Z, const double* alpha,
                     const double* beta, bool x_init) {
  if (dtype == BKTS_F64)
    BKTS_RK_DISPATCH(k, (rk_cg_xp_t<double, KP>(ctx, N, X, P, Z, alpha, beta, x_init)));
  else
    BKTS_RK_DISPATCH(k, (rk_cg_xp_t<float, KP>(ctx, N, X, P, Z, alpha, beta, x_init)));
}

template <typename T, int KP>
static void rk_cg_pupdate_t(bkts_ctx ctx, int64_t N, void* P, const void* R, const double* beta, const double* dinv) {
  const int64_t nb = rk_grid(ctx, rk_cg_pupdate_kernel<T, KP>, N);
  ProfScope prof(ctx, BKTS_K_CG_PUPDATE, (beta ? 3.0 : 2.0) * N * KP * sizeof(T) + (dinv ? 8.0 * N : 0.0));
  launch(ctx, (rk_cg_pupdate_kernel<T, KP>), dim3(nb), dim3(256), 0, N, static_cast<T*>(P),
                     static_cast<const T*>(R), beta, dinv);
  BKTS_HIP(hipGetLastError());
}

void rk_cg_pupdate(bkts_ctx ctx, int dtype, int64_t N, int k, void* P, const void* R, const double* beta,
                   const double* dinv) {
  if (dtype == BKTS_F64)
    BKTS_RK_DISPATCH(k, (rk_cg_pupdate_t<double, KP>(ctx, N, P, R, beta, dinv)));
  else
    BKTS_RK_DISPATCH(k, (rk_cg_pupdate_t<float, KP>(ctx, N, P, R, beta, dinv)));
}

template <typename T, int KP>
static void rk_gram_t(bkts_ctx ctx, int64_t N, const void* X, const void* Y, double* G) {
  const int64_t nb = rk_grid(ctx, rk_gram_kernel<T, KP>, N);
  double* part = ctx->ws.get<double>("rk_gram_part", (size_t)KP * KP * nb);
  ProfScope prof(ctx, BKTS_K_GRAM, 2.0 * N * KP * sizeof(T));
  launch(ctx, (rk_gram_kernel<T, KP>), dim3(nb), dim3(256), 0, N, static_cast<const T*>(X),
                     static_cast<const T*>(Y), part);
  BKTS_HIP(hipGetLastError());
  prof.end();
  finalize_gram(ctx, part, (int)nb, KP, KP, G);
}

template <typename T, int KP>
static void rk_gram2_t(bkts_ctx ctx, int64_t N, const void* X1, const void* X2, const void* Y, double* G1,
                       double* G2) {
  const int64_t nb = rk_grid(ctx, rk_gram2_kernel<T, KP>, N);
  double* part = ctx->ws.get<double>("rk_gram2_part", (size_t)2 * KP * KP * nb);
  ProfScope prof(ctx, BKTS_K_GRAM, 3.0 * N * KP * sizeof(T));
  launch(ctx, (rk_gram2_kernel<T, KP>), dim3(nb), dim3(256), 0, N, static_cast<const T*>(X1),
         static_cast<const T*>(X2), static_cast<const T*>(Y), part);
  BKTS_HIP(hipGetLastError());
  prof.end();
  const FoldSet sets[2] = {{part, KP, 0, G1}, {part + (size_t)KP * KP * nb, KP, 0, G2}};
  finalize_sets(ctx, (int)nb, KP, sets, 2);
}

void rk_gram2(bkts_ctx ctx, int dtype, int64_t N, int k, const void* X1, const void* X2, const void* Y, double* G1,
              double* G2) {
  if (dtype == BKTS_F64)
    BKTS_RK_DISPATCH(k, (rk_gram2_t<double, KP>(ctx, N, X1, X2, Y, G1, G2)));
  else
    BKTS_RK_DISPATCH(k, (rk_gram2_t<float, KP>(ctx, N, X1, X2, Y, G1, G2)));
}

void rk_gram(bkts_ctx ctx, int dtype, int64_t N, int k, const void* X, const void* Y, double* G) {
  if (dtype == BKTS_F64)
    BKTS_RK_DISPATCH(k, (rk_gram_t<double, KP>(ctx, N, X, Y, G)));
  else
    BKTS_RK_DISPATCH(k, (rk_gram_t<float, KP>(ctx, N, X, Y, G)));
}

template <typename T, int KP>
static void rk_rmul_t(bkts_ctx ctx, int64_t N, const void* X, const double* C, double c0, double c1, void* Y) {
  const int64_t nb = rk_grid(ctx, rk_rmul_kernel<T, KP>, N);
  ProfScope prof(ctx, BKTS_K_OTHER, (c0 != 0.0 ? 3.0 : 2.0) * N * KP * sizeof(T));
  launch(ctx, (rk_rmul_kernel<T, KP>), dim3(nb), dim3(256), 0, N, static_cast<const T*>(X), C, c0,
                     c1, static_cast<T*>(Y));
  BKTS_HIP(hipGetLastError());
}

void rk_rmul(bkts_ctx ctx, int dtype, int64_t N, int k, const void* X, const double* C, double c0, double c1,
             void* Y) {
  if (dtype == BKTS_F64)
    BKTS_RK_DISPATCH(k, (rk_rmul_t<double, KP>(ctx, N, X, C, c0, c1, Y)));
  else
    BKTS_RK_DISPATCH(k, (rk_rmul_t<float, KP>(ctx, N, X, C, c0, c1, Y)));
}

template <typename S, typename D, int KP>
static void rk_cast_t(bkts_ctx ctx, int64_t N, const void* src, void* dst, const double* s, bool invert,
                      bool accumulate, bool norm2, double coef) {
  launch(ctx, (rk_cast_kernel<S, D, KP>), dim3((unsigned)((N + 255) / 256)), dim3(256), 0, N,
         static_cast<const S*>(src), static_cast<D*>(dst), s, (int)invert, (int)accumulate, (int)norm2, coef);
  BKTS_HIP(hipGetLastError());
}

bool rk_cast(bkts_ctx ctx, int64_t N, int k, int src_t, const void* src, int dst_t, void* dst, const double* s,
             bool invert, bool accumulate, bool norm2, double coef) {
  auto aligned = [](const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; };
  if (!rk_eligible(k) || !aligned(src) || !aligned(dst) || N >= ((int64_t)1 << 38)) return false;
  if (src_t == BKTS_F64 && dst_t == BKTS_F32)
    BKTS_RK_DISPATCH(k, (rk_cast_t<double, float, KP>(ctx, N, src, dst, s, invert, accumulate, norm2, coef)));
  else if (src_t == BKTS_F32 && dst_t == BKTS_F64)
    BKTS_RK_DISPATCH(k, (rk_cast_t<float, double, KP>(ctx, N, src, dst, s, invert, accumulate, norm2, coef)));
  else
    return false;
  return true;
}

}  // namespace bkts

// FP32 block-CG kernels for wide blocks (8 < KP <= 32 columns, padded to KP = 16 NB) on the FP32
// matrix cores of gfx950 (v_mfma_f32_16x16x4f32).  The right multiplications by k x k coefficient
// matrices and the k x k Gram products are dense contractions, so they run on MFMA while the
// blocks stream through once.
//
// Operand layouts of v_mfma_f32_16x16x4f32 (checked on the device):
//   A (16 x 4): lane l holds A[l % 16][l / 16]
//   B (4 x 16): lane l holds B[l / 16][l % 16]
//   D (16 x 16, four registers v): lane l holds D[4 (l / 16) + v][l % 16]
// A 16-row tile is kept in the D layout: lane (g = l/16, c = l%16), register r holds row 4g + r,
// column 16 cb + c.  Loads and stores of that layout are coalesced (16 lanes cover 64 contiguous
// bytes of one row), it is directly the accumulator of `tile x (k x k)` products, and a Gram
// X^T Y over the tile is four MFMAs (one per register r) with both operands taken as they are.
// Only the A operand of a right multiplication (row l%16, column 4 kb + l/16) is a transposed
// read; it comes from a per-wave LDS copy of the tile.
//
// Gram partial sums are formed in FP32 over one 16-row tile and accumulated in FP64 across
// tiles; the k x k coefficients are FP64 in memory and rounded to FP32 for the products.
//
// The bodies take explicit pointers and a tile range, so the single-solve kernels and the grouped
// serving kernels run the same code.
#include "devcommon.hpp"
#include "internal.hpp"
#include "serve.hpp"
#include "wide.hpp"

namespace bkts {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f4 mfma32(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

template <int NB>
struct WG {
  static constexpr int KP = 16 * NB;
  static constexpr int LDT = KP + 1;     // LDS row stride (floats) of a tile copy
  static constexpr int TILE = 16 * LDT;  // floats per tile copy
};

template <int NB>
__device__ __forceinline__ void wload(const float* __restrict__ M, int64_t N, int k, int64_t row0,
                                      float (&d)[NB][4]) {
  const int l = threadIdx.x & 63, g = l >> 4, c = l & 15;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int64_t row = row0 + 4 * g + r;
#pragma unroll
    for (int cb = 0; cb < NB; ++cb) {
      const int col = 16 * cb + c;
      d[cb][r] = (row < N && col < k) ? M[row * k + col] : 0.f;
    }
  }
}

template <int NB>
__device__ __forceinline__ void wstore(float* __restrict__ M, int64_t N, int k, int64_t row0, const f4 (&d)[NB],
                                       float sign) {
  const int l = threadIdx.x & 63, g = l >> 4, c = l & 15;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int64_t row = row0 + 4 * g + r;
#pragma unroll
    for (int cb = 0; cb < NB; ++cb) {
      const int col = 16 * cb + c;
      if (row < N && col < k) M[row * k + col] = sign * d[cb][r];
    }
  }
}

// Per-row Jacobi factors of the lane's four rows.
__device__ __forceinline__ void wdinv(const double* dinv, int64_t N, int64_t row0, float (&dv)[4]) {
  const int g = (threadIdx.x & 63) >> 4;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int64_t row = row0 + 4 * g + r;
    dv[r] = (dinv && row < N) ? (float)dinv[row] : 1.f;
  }
}

template <int NB>
__device__ __forceinline__ void wlds_put(float* lds, const float (&d)[NB][4]) {
  const int l = threadIdx.x & 63, g = l >> 4, c = l & 15;
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int cb = 0; cb < NB; ++cb) lds[(4 * g + r) * WG<NB>::LDT + 16 * cb + c] = d[cb][r];
}

template <int NB>
__device__ __forceinline__ void wlds_afrag(const float* lds, float (&a)[4 * NB]) {
  const int l = threadIdx.x & 63;
#pragma unroll
  for (int kb = 0; kb < 4 * NB; ++kb) a[kb] = lds[(l & 15) * WG<NB>::LDT + 4 * kb + (l >> 4)];
}

// B fragments of a k x k FP64 matrix: f[kb][cb] = M[4 kb + l/16][16 cb + l%16] (zero outside k).
template <int NB>
__device__ __forceinline__ void wbfrag(const double* M, int k, float (&f)[4 * NB][NB]) {
  const int l = threadIdx.x & 63, g = l >> 4, c = l & 15;
#pragma unroll
  for (int kb = 0; kb < 4 * NB; ++kb)
#pragma unroll
    for (int cb = 0; cb < NB; ++cb) {
      const int r = 4 * kb + g, col = 16 * cb + c;
      f[kb][cb] = (M && r < k && col < k) ? (float)M[r * k + col] : 0.f;
    }
}

// out[cb] = T_tile(rows x KP) * M + cin[cb], T's A fragments in a.
template <int NB>
__device__ __forceinline__ void wrmul(const float (&a)[4 * NB], const float (&f)[4 * NB][NB], const float (&cin)[NB][4],
                                      float csign, f4 (&out)[NB]) {
#pragma unroll
  for (int cb = 0; cb < NB; ++cb) {
    f4 acc = f4{csign * cin[cb][0], csign * cin[cb][1], csign * cin[cb][2], csign * cin[cb][3]};
#pragma unroll
    for (int kb = 0; kb < 4 * NB; ++kb) acc = mfma32(a[kb], f[kb][cb], acc);
    out[cb] = acc;
  }
}

// acc64 += X_tile^T Y_tile (FP32 MFMA over the tile, FP64 across tiles).
template <int NB>
__device__ __forceinline__ void wgram(const float (&x)[NB][4], const float (&y)[NB][4], double (&acc)[NB][NB][4]) {
#pragma unroll
  for (int ia = 0; ia < NB; ++ia)
#pragma unroll
    for (int jb = 0; jb < NB; ++jb) {
      f4 t = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int r = 0; r < 4; ++r) t = mfma32(x[ia][r], y[jb][r], t);
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[ia][jb][v] += (double)t[v];
    }
}

// Fold the 4 waves' k x k accumulators (D layout) into partials[(a*KP + b) * nslots + slot].
// `red` holds 4*KP*KP doubles.  Workgroup barriers inside.
template <int NB>
__device__ void wfold(const double (&acc)[NB][NB][4], double* red, double* partials, int64_t nslots, int64_t slot) {
  constexpr int KP = 16 * NB;
  const int l = threadIdx.x & 63, w = threadIdx.x >> 6, g = l >> 4, c = l & 15;
  __syncthreads();
#pragma unroll
  for (int ia = 0; ia < NB; ++ia)
#pragma unroll
    for (int jb = 0; jb < NB; ++jb)
#pragma unroll
      for (int v = 0; v < 4; ++v) red[w * KP * KP + (16 * ia + 4 * g + v) * KP + 16 * jb + c] = acc[ia][jb][v];
  __syncthreads();
  for (int e = threadIdx.x; e < KP * KP; e += dev::kThreads)
    partials[(int64_t)e * nslots + slot] = ((red[e] + red[KP * KP + e]) + red[2 * KP * KP + e]) + red[3 * KP * KP + e];
  __syncthreads();
}

// Column sums of squares: per-lane s[cb] over its rows, folded over lane groups and waves.
template <int NB>
__device__ void wfold_cols(double (&s)[NB], double* red, double* partials, int64_t nslots, int64_t slot) {
  constexpr int KP = 16 * NB;
  const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int cb = 0; cb < NB; ++cb) {
    s[cb] += __shfl_xor(s[cb], 16);
    s[cb] += __shfl_xor(s[cb], 32);
  }
  __syncthreads();
  if (l < 16) {
#pragma unroll
    for (int cb = 0; cb < NB; ++cb) red[w * KP + 16 * cb + l] = s[cb];
  }
  __syncthreads();
  if (threadIdx.x < KP) {
    const int e = threadIdx.x;
    partials[(int64_t)e * nslots + slot] = ((red[e] + red[KP + e]) + red[2 * KP + e]) + red[3 * KP + e];
  }
  __syncthreads();
}

template <int NB>
constexpr int wide_lds_floats() {
  // per-wave P and Q tile copies, or the fold buffer (4 KP^2 doubles)
  return (8 * WG<NB>::TILE > 8 * 16 * NB * 16 * NB) ? 8 * WG<NB>::TILE : 8 * 16 * NB * 16 * NB;
}

// Tiles [t0, t1) of a workgroup are dealt to its 4 waves round-robin.
struct TileRange {
  int64_t t0, t1;
};

__device__ __forceinline__ TileRange slot_tiles(int64_t ntiles, int64_t nslots, int64_t slot) {
  const int64_t per = (ntiles + nslots - 1) / nslots;
  TileRange r;
  r.t0 = slot * per < ntiles ? slot * per : ntiles;
  r.t1 = (slot + 1) * per < ntiles ? (slot + 1) * per : ntiles;
  return r;
}

// X += P alpha; R -= Q alpha; Z = Dinv R; gamma = R^T Z; T = Q^T Z; nrm = diag(R^T R).
template <int NB>
__device__ void w_update_body(const WideArgs& a, int64_t nslots, int64_t slot, float* lds_f) {
  using G = WG<NB>;
  const int w = threadIdx.x >> 6;
  float* Pl = lds_f + (2 * w) * G::TILE;
  float* Ql = Pl + G::TILE;
  float af[4 * NB][NB];
  wbfrag<NB>(a.coef, a.k, af);
  double gam[NB][NB][4], tac[NB][NB][4], nrm[NB];
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    nrm[i] = 0.0;
#pragma unroll
    for (int j = 0; j < NB; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) gam[i][j][v] = tac[i][j][v] = 0.0;
  }
  const int64_t ntiles = (a.N + 15) / 16;
  const TileRange tr = slot_tiles(ntiles, nslots, slot);
  // NB = 1: the next tile's loads are issued before the current tile is computed (two in flight)
  float pd[NB][4], qd[NB][4], xd[NB][4], rd[NB][4], dv[4];
  int64_t t = tr.t0 + w;
  if (NB == 1 && t < tr.t1) {
    wload<NB>(a.P, a.N, a.k, 16 * t, pd);
    wload<NB>(a.Q, a.N, a.k, 16 * t, qd);
    wload<NB>(a.X, a.N, a.k, 16 * t, xd);
    wload<NB>(a.R, a.N, a.k, 16 * t, rd);
    wdinv(a.dinv, a.N, 16 * t, dv);
  }
  for (; t < tr.t1; t += 4) {
    const int64_t row0 = 16 * t;
    if (NB != 1) {
      wload<NB>(a.P, a.N, a.k, row0, pd);
      wload<NB>(a.Q, a.N, a.k, row0, qd);
      wload<NB>(a.X, a.N, a.k, row0, xd);
      wload<NB>(a.R, a.N, a.k, row0, rd);
      wdinv(a.dinv, a.N, row0, dv);
    }
    // prefetch only where registers allow (NB = 2 would drop to one wave per SIMD)
    const bool more = NB == 1 && t + 4 < tr.t1;
    float pn_[NB][4], qn_[NB][4], xn_[NB][4], rn_[NB][4], dn_[4];
    if (more) {
      wload<NB>(a.P, a.N, a.k, row0 + 64, pn_);
      wload<NB>(a.Q, a.N, a.k, row0 + 64, qn_);
      wload<NB>(a.X, a.N, a.k, row0 + 64, xn_);
      wload<NB>(a.R, a.N, a.k, row0 + 64, rn_);
      wdinv(a.dinv, a.N, row0 + 64, dn_);
    }
    wlds_put<NB>(Pl, pd);
    wlds_put<NB>(Ql, qd);
    __builtin_amdgcn_wave_barrier();
    float pa[4 * NB], qa[4 * NB];
    wlds_afrag<NB>(Pl, pa);
    wlds_afrag<NB>(Ql, qa);
    f4 xn[NB], rn[NB];
    wrmul<NB>(pa, af, xd, 1.f, xn);   // X + P alpha
    wrmul<NB>(qa, af, rd, -1.f, rn);  // Q alpha - R
    wstore<NB>(a.X, a.N, a.k, row0, xn, 1.f);
    wstore<NB>(a.R, a.N, a.k, row0, rn, -1.f);
    float rr[NB][4], z[NB][4];
#pragma unroll
    for (int cb = 0; cb < NB; ++cb)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        rr[cb][r] = -rn[cb][r];
        z[cb][r] = rr[cb][r] * dv[r];
        nrm[cb] = fma((double)rr[cb][r], (double)rr[cb][r], nrm[cb]);
      }
    wgram<NB>(rr, z, gam);
    wgram<NB>(qd, z, tac);
    __builtin_amdgcn_wave_barrier();
    if (more) {
#pragma unroll
      for (int cb = 0; cb < NB; ++cb)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          pd[cb][r] = pn_[cb][r];
          qd[cb][r] = qn_[cb][r];
          xd[cb][r] = xn_[cb][r];
          rd[cb][r] = rn_[cb][r];
        }
#pragma unroll
      for (int r = 0; r < 4; ++r) dv[r] = dn_[r];
    }
  }
  double* red = reinterpret_cast<double*>(lds_f);
  wfold<NB>(gam, red, a.pg, nslots, slot);
  wfold<NB>(tac, red, a.pt, nslots, slot);
  wfold_cols<NB>(nrm, red, a.pn, nslots, slot);
}

// P = Dinv R + P beta  (coef == null: P = Dinv R)
template <int NB>
__device__ void w_pupdate_body(const WideArgs& a, int64_t nslots, int64_t slot, float* lds_f) {
  using G = WG<NB>;
  const int w = threadIdx.x >> 6;
  float* Pl = lds_f + (2 * w) * G::TILE;
  float bf[4 * NB][NB];
  wbfrag<NB>(a.coef, a.k, bf);
  const int64_t ntiles = (a.N + 15) / 16;
  const TileRange tr = slot_tiles(ntiles, nslots, slot);
  for (int64_t t = tr.t0 + w; t < tr.t1; t += 4) {
    const int64_t row0 = 16 * t;
    float pd[NB][4], zd[NB][4], dv[4];
    wload<NB>(a.R, a.N, a.k, row0, zd);
    wdinv(a.dinv, a.N, row0, dv);
#pragma unroll
    for (int cb = 0; cb < NB; ++cb)
#pragma unroll
      for (int r = 0; r < 4; ++r) zd[cb][r] *= dv[r];
    f4 pn[NB];
    if (a.coef) {
      wload<NB>(a.P, a.N, a.k, row0, pd);
      wlds_put<NB>(Pl, pd);
      __builtin_amdgcn_wave_barrier();
      float pa[4 * NB];
      wlds_afrag<NB>(Pl, pa);
      wrmul<NB>(pa, bf, zd, 1.f, pn);
    } else {
#pragma unroll
      for (int cb = 0; cb < NB; ++cb) pn[cb] = f4{zd[cb][0], zd[cb][1], zd[cb][2], zd[cb][3]};
    }
    wstore<NB>(a.P, a.N, a.k, row0, pn, 1.f);
    __builtin_amdgcn_wave_barrier();
  }
}

// Q = alpha P + beta K P (CSR, FP32 values and accumulation) and G = P^T Q.
template <int NB>
__device__ void w_spmm_gram_body(const WideArgs& a, int64_t nslots, int64_t slot, float* lds_f) {
  const int w = threadIdx.x >> 6;
  const int l = threadIdx.x & 63, g = l >> 4, c = l & 15;
  double gacc[NB][NB][4];
#pragma unroll
  for (int i = 0; i < NB; ++i)
#pragma unroll
    for (int j = 0; j < NB; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) gacc[i][j][v] = 0.0;
  const float fa = (float)a.sa, fb = (float)a.sb;
  const int64_t ntiles = (a.N + 15) / 16;
  const TileRange tr = slot_tiles(ntiles, nslots, slot);
  for (int64_t t = tr.t0 + w; t < tr.t1; t += 4) {
    const int64_t row0 = 16 * t;
    float pd[NB][4], qd[NB][4];
    wload<NB>(a.P, a.N, a.k, row0, pd);
    int32_t beg[4], len[4];
    int maxlen = 0;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t row = row0 + 4 * g + r;
      beg[r] = row < a.N ? a.rowptr[row] : 0;
      len[r] = row < a.N ? a.rowptr[row + 1] - beg[r] : 0;
      maxlen = len[r] > maxlen ? len[r] : maxlen;
    }
    float s[NB][4];
#pragma unroll
    for (int cb = 0; cb < NB; ++cb)
#pragma unroll
      for (int r = 0; r < 4; ++r) s[cb][r] = 0.f;
    // all entry loads of a chunk first, then all gathers: two dependent round trips per chunk
    constexpr int U = 8;
    for (int j0 = 0; j0 < maxlen; j0 += U) {
      float v[4][U];
      int32_t ci[4][U];
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const bool ok = j0 + u < len[r];
          v[r][u] = ok ? a.val[beg[r] + j0 + u] : 0.f;
          ci[r][u] = ok ? a.col[beg[r] + j0 + u] : 0;
        }
#pragma unroll
      for (int cb = 0; cb < NB; ++cb) {
        const int col = 16 * cb + c < a.k ? 16 * cb + c : 0;
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
          for (int u = 0; u < U; ++u) s[cb][r] = fmaf(v[r][u], a.P[(int64_t)ci[r][u] * a.k + col], s[cb][r]);
      }
    }
#pragma unroll
    for (int cb = 0; cb < NB; ++cb) {
      const int col = 16 * cb + c;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = row0 + 4 * g + r;
        const bool ok = row < a.N && col < a.k;
        qd[cb][r] = ok ? fmaf(fa, pd[cb][r], fb * s[cb][r]) : 0.f;
        if (ok) a.Q[row * a.k + col] = qd[cb][r];
      }
    }
    wgram<NB>(pd, qd, gacc);
  }
  (void)w;
  wfold<NB>(gacc, reinterpret_cast<double*>(lds_f), a.pg, nslots, slot);
}

// G = X^T Y
template <int NB>
__device__ void w_gram_body(const WideArgs& a, int64_t nslots, int64_t slot, float* lds_f) {
  const int w = threadIdx.x >> 6;
  double gacc[NB][NB][4];
#pragma unroll
  for (int i = 0; i < NB; ++i)
#pragma unroll
    for (int j = 0; j < NB; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) gacc[i][j][v] = 0.0;
  const int64_t ntiles = (a.N + 15) / 16;
  const TileRange tr = slot_tiles(ntiles, nslots, slot);
  for (int64_t t = tr.t0 + w; t < tr.t1; t += 4) {
    float xd[NB][4], yd[NB][4];
    wload<NB>(a.X, a.N, a.k, 16 * t, xd);
    wload<NB>(a.P, a.N, a.k, 16 * t, yd);
    wgram<NB>(xd, yd, gacc);
  }
  wfold<NB>(gacc, reinterpret_cast<double*>(lds_f), a.pg, nslots, slot);
}

// ------------------------------------------------------------------ single-solve kernels

template <int NB>
__global__ __launch_bounds__(256) void w_gram_kernel(WideArgs a) {
  __shared__ __align__(16) float lds[wide_lds_floats<NB>()];
  w_gram_body<NB>(a, gridDim.x, dev::xcd_slot(blockIdx.x, gridDim.x), lds);
}

template <int NB>
__global__ __launch_bounds__(256) void w_update_kernel(WideArgs a) {
  __shared__ __align__(16) float lds[wide_lds_floats<NB>()];
  w_update_body<NB>(a, gridDim.x, dev::xcd_slot(blockIdx.x, gridDim.x), lds);
}

template <int NB>
__global__ __launch_bounds__(256) void w_pupdate_kernel(WideArgs a) {
  __shared__ __align__(16) float lds[wide_lds_floats<NB>()];
  w_pupdate_body<NB>(a, gridDim.x, dev::xcd_slot(blockIdx.x, gridDim.x), lds);
}

template <int NB>
__global__ __launch_bounds__(256) void w_spmm_gram_kernel(WideArgs a) {
  __shared__ __align__(16) float lds[wide_lds_floats<NB>()];
  w_spmm_gram_body<NB>(a, gridDim.x, dev::xcd_slot(blockIdx.x, gridDim.x), lds);
}

// ------------------------------------------------------------------ grouped kernels

__device__ __forceinline__ int find_job(const int* first, int n, int b) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (first[mid] <= b) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

__device__ __forceinline__ WideArgs job_args(const GJob& J, int op) {
  WideArgs a{};
  a.N = J.N;
  a.k = J.k;
  a.X = J.X;
  a.P = J.P;
  a.Q = J.Q;
  a.R = J.R;
  a.dinv = J.dinv;
  a.rowptr = J.rowptr;
  a.col = J.col;
  a.val = J.val;
  a.sa = J.a;
  a.sb = J.b;
  a.pg = J.pg;
  a.pt = J.pt;
  a.pn = J.pn;
  a.coef = op == 0 ? J.alpha : J.beta;
  return a;
}

template <int NB, int OP>
__global__ __launch_bounds__(256) void gw_kernel(const GJob* __restrict__ jobs, const int* ids, const int* first,
                                                 int n) {
  __shared__ __align__(16) float lds[wide_lds_floats<NB>()];
  const int gi = find_job(first, n, blockIdx.x);
  const GJob& J = jobs[ids[gi]];
  const int64_t slot = blockIdx.x - first[gi];
  if constexpr (OP == 0) w_spmm_gram_body<NB>(job_args(J, 0), J.nslots, slot, lds);
  if constexpr (OP == 1) w_update_body<NB>(job_args(J, 0), J.nslots, slot, lds);
  if constexpr (OP == 2) w_pupdate_body<NB>(job_args(J, 1), J.nslots, slot, lds);
}

int64_t wide_blocks(bkts_ctx ctx, const void* kern, int64_t ntiles) {
  const int64_t cap = (int64_t)blocks_per_cu(kern) * ctx->num_cu;
  const int64_t want = (ntiles + 3) / 4;  // at least one tile per wave
  int64_t nb = want < cap ? want : cap;
  return nb < 1 ? 1 : nb;
}

}  // namespace

bool wide_eligible(int dtype, int k) { return dtype == BKTS_F32 && k >= 5 && k <= 32; }

int wide_kp(int k) { return k <= 16 ? 16 : 32; }

#define BKTS_WNB(k, CALL)                                 \
  do {                                                    \
    if ((k) <= 16) { constexpr int NB = 1; CALL; }        \
    else { constexpr int NB = 2; CALL; }                  \
  } while (0)

void w_cg_update(bkts_ctx ctx, int64_t N, int k, float* X, const float* P, float* R, const float* Q,
                 const double* alpha, const double* dinv, double* gamma, double* Tm, double* nrm,
                 const CgTail* tail) {
  const int KP = wide_kp(k);
  const int64_t nb = wide_blocks(ctx, k <= 16 ? (const void*)w_update_kernel<1> : (const void*)w_update_kernel<2>,
                                 (N + 15) / 16);
  const size_t np = (size_t)KP * KP * nb;
  WideArgs a{};
  a.N = N;
  a.k = k;
  a.X = X;
  a.P = const_cast<float*>(P);
  a.R = R;
  a.Q = const_cast<float*>(Q);
  a.coef = alpha;
  a.dinv = dinv;
  a.pg = ctx->ws.get<double>("w_upd", 2 * np + (size_t)KP * nb);  // [gamma | T | nrm] entries
  a.pt = a.pg + np;
  a.pn = a.pt + np;
  ProfScope prof(ctx, BKTS_K_CG_UPDATE, 24.0 * N * k + (dinv ? 8.0 * N : 0.0));
  BKTS_WNB(k, launch(ctx, w_update_kernel<NB>, dim3(nb), dim3(256), 0, a));
  BKTS_HIP(hipGetLastError());
  prof.end();
  if (tail) return fold_solve(ctx, 1, KP, k, a.pg, nb, *tail);
  const FoldSet sets[3] = {{a.pg, KP, 0, gamma}, {a.pt, KP, 0, Tm}, {a.pn, KP, 1, nrm}};
  finalize_sets(ctx, (int)nb, k, sets, 3);
}

void w_cg_pupdate(bkts_ctx ctx, int64_t N, int k, float* P, const float* R, const double* beta, const double* dinv) {
  const int64_t nb = wide_blocks(ctx, k <= 16 ? (const void*)w_pupdate_kernel<1> : (const void*)w_pupdate_kernel<2>,
                                 (N + 15) / 16);
  WideArgs a{};
  a.N = N;
  a.k = k;
  a.P = P;
  a.R = const_cast<float*>(R);
  a.coef = beta;
  a.dinv = dinv;
  ProfScope prof(ctx, BKTS_K_CG_PUPDATE, (beta ? 12.0 : 8.0) * N * k + (dinv ? 8.0 * N : 0.0));
  BKTS_WNB(k, launch(ctx, w_pupdate_kernel<NB>, dim3(nb), dim3(256), 0, a));
  BKTS_HIP(hipGetLastError());
}

void w_spmm_gram(bkts_ctx ctx, const bkts_op_s& op, int k, double alpha, const float* P, double beta, float* Q,
                 double* G) {
  const int KP = wide_kp(k);
  const int64_t N = op.N;
  const int64_t nb = wide_blocks(
      ctx, k <= 16 ? (const void*)w_spmm_gram_kernel<1> : (const void*)w_spmm_gram_kernel<2>, (N + 15) / 16);
  WideArgs a{};
  a.N = N;
  a.k = k;
  a.P = const_cast<float*>(P);
  a.Q = Q;
  a.rowptr = op.rowptr.as<int32_t>();
  a.col = op.col.as<int32_t>();
  a.val = op.val32.as<float>();
  a.sa = alpha;
  a.sb = beta;
  a.pg = ctx->ws.get<double>("w_sg", (size_t)KP * KP * nb);
  ProfScope prof(ctx, BKTS_K_SPMM, op.nnz * 8.0 + 4.0 * (N + 1) + 8.0 * N * k);
  BKTS_WNB(k, launch(ctx, w_spmm_gram_kernel<NB>, dim3(nb), dim3(256), 0, a));
  BKTS_HIP(hipGetLastError());
  prof.end();
  finalize_gram(ctx, a.pg, (int)nb, k, KP, G);
}

void w_gram(bkts_ctx ctx, int64_t N, int k, const float* X, const float* Y, double* G, const CgTail* tail) {
  const int KP = wide_kp(k);
  const int64_t nb =
      wide_blocks(ctx, k <= 16 ? (const void*)w_gram_kernel<1> : (const void*)w_gram_kernel<2>, (N + 15) / 16);
  WideArgs a{};
  a.N = N;
  a.k = k;
  a.X = const_cast<float*>(X);
  a.P = const_cast<float*>(Y);
  a.pg = ctx->ws.get<double>("w_gram", (size_t)KP * KP * nb);
  ProfScope prof(ctx, BKTS_K_GRAM, 8.0 * N * k);
  BKTS_WNB(k, launch(ctx, w_gram_kernel<NB>, dim3(nb), dim3(256), 0, a));
  BKTS_HIP(hipGetLastError());
  prof.end();
  if (tail) return fold_solve(ctx, 0, KP, k, a.pg, nb, *tail);
  finalize_gram(ctx, a.pg, (int)nb, k, KP, G);
}

void gw_spmm_gram(bkts_ctx ctx, int nb, const GJob* jobs, GList l) {
  if (l.n == 0 || l.total == 0) return;
  BKTS_WNB(16 * nb, (launch(ctx, gw_kernel<NB, 0>, dim3(l.total), dim3(256), 0, jobs, l.ids, l.first, l.n)));
  BKTS_HIP(hipGetLastError());
}

void gw_update(bkts_ctx ctx, int nb, const GJob* jobs, GList l) {
  if (l.n == 0 || l.total == 0) return;
  BKTS_WNB(16 * nb, (launch(ctx, gw_kernel<NB, 1>, dim3(l.total), dim3(256), 0, jobs, l.ids, l.first, l.n)));
  BKTS_HIP(hipGetLastError());
}

void gw_pupdate(bkts_ctx ctx, int nb, const GJob* jobs, GList l) {
  if (l.n == 0 || l.total == 0) return;
  BKTS_WNB(16 * nb, (launch(ctx, gw_kernel<NB, 2>, dim3(l.total), dim3(256), 0, jobs, l.ids, l.first, l.n)));
  BKTS_HIP(hipGetLastError());
}

}  // namespace bkts

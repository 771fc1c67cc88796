// Block-vector kernels for 8 <= k <= 32 built on the FP64 matrix cores of gfx950
// (v_mfma_f64_16x16x4f64): the k x k Gram products X^T Y and the right multiplications by k x k
// coefficient matrices are dense contractions, so they run on MFMA while the data streams through
// once.  Blocks are padded to KP = 16*NB columns (NB = 1 or 2); padding columns load as zero.
//
// Operand layouts of v_mfma_f64_16x16x4f64 (checked on the device):
//   A (16 x 4): lane l holds A[l % 16][l / 16]
//   B (4 x 16): lane l holds B[l / 16][l % 16]
//   D (16 x 16, four registers v): lane l holds D[4v + l/16][l % 16]
// so register v of an accumulator is the natural row-major layout of rows 4v..4v+3 (lane l <->
// row 4v + l/16, column l % 16).  Consequences used below:
//   * Gram G += X^T Y over a quad of rows is ONE instruction with A = X, B = Y taken straight
//     from coalesced row-major loads of that quad (no shuffles, no LDS);
//   * a 16-row tile times a k x k matrix accumulates into registers that are again coalesced
//     row-major quads; only its A operand (row l%16, column 4kb + l/16) is a transposed read,
//     served from a per-wave LDS copy of the tile.
// Every wave owns a contiguous range of 16-row tiles (workgroups remapped per XCD); the k x k
// accumulators of the 4 waves of a workgroup are folded in a fixed order into one partial per
// workgroup, which finalize_partials() sums in a fixed order (bitwise reproducible).
#include <algorithm>

#include "devcommon.hpp"
#include "internal.hpp"

namespace bkts {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ d4 mfma(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ d4 zero4() { return d4{0.0, 0.0, 0.0, 0.0}; }

// FP32 matrix cores (v_mfma_f32_16x16x4f32): same A and B layouts as the FP64 instruction; its D
// layout differs: lane l, register v holds D[4 (l / 16) + v][l % 16].
typedef float f4m __attribute__((ext_vector_type(4)));
__device__ __forceinline__ f4m mfma32(float a, float b, f4m c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

template <int NB>
struct MGeom {
  static constexpr int KP = 16 * NB;
  static constexpr int LDT = KP + 1;            // LDS row stride (doubles) of a 16-row tile
  static constexpr int TILE = 16 * LDT;         // doubles per tile copy
};

struct WaveRange {
  int64_t begin, end;  // [begin, end) in units (tiles or quads)
};

// Contiguous range of `nunits` work units owned by wave `w` of the (XCD-remapped) workgroup.
__device__ __forceinline__ WaveRange wave_range(int64_t nunits) {
  const int64_t slot = dev::xcd_slot(blockIdx.x, gridDim.x);
  const int64_t nw = (int64_t)gridDim.x * 4;
  const int64_t w = slot * 4 + (threadIdx.x >> 6);
  const int64_t per = (nunits + nw - 1) / nw;
  WaveRange r;
  r.begin = w * per < nunits ? w * per : nunits;
  r.end = (w + 1) * per < nunits ? (w + 1) * per : nunits;
  return r;
}

template <typename T>
__device__ __forceinline__ double ldz(const T* p, bool ok) {
  return ok ? static_cast<double>(*p) : 0.0;
}

// Fold the per-wave k x k accumulators acc[ia][jb] (D layout) of the 4 waves into one partial per
// workgroup: partials[e * nslots + slot], e = a*KP + b.  `red` holds 4*KP*KP doubles.  Barriers inside.
template <int NB>
__device__ void fold_kxk(d4 (&acc)[NB][NB], double* red, double* partials) {
  constexpr int KP = 16 * NB;
  const int l = threadIdx.x & 63, w = threadIdx.x >> 6, g = l >> 4, c = l & 15;
  __syncthreads();
#pragma unroll
  for (int ia = 0; ia < NB; ++ia)
#pragma unroll
    for (int jb = 0; jb < NB; ++jb)
#pragma unroll
      for (int v = 0; v < 4; ++v) red[w * KP * KP + (16 * ia + 4 * v + g) * KP + 16 * jb + c] = acc[ia][jb][v];
  __syncthreads();
  const int64_t slot = dev::xcd_slot(blockIdx.x, gridDim.x);
  for (int e = threadIdx.x; e < KP * KP; e += dev::kThreads) {
    const double s = ((red[e] + red[KP * KP + e]) + red[2 * KP * KP + e]) + red[3 * KP * KP + e];
    partials[(int64_t)e * gridDim.x + slot] = s;
  }
  __syncthreads();
}

// fold_kxk for accumulators in the FP32 D layout (register v of lane l is row 4 (l / 16) + v).
template <int NB>
__device__ void fold_kxk32(d4 (&acc)[NB][NB], double* red, double* partials) {
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
  const int64_t slot = dev::xcd_slot(blockIdx.x, gridDim.x);
  for (int e = threadIdx.x; e < KP * KP; e += dev::kThreads) {
    const double s = ((red[e] + red[KP * KP + e]) + red[2 * KP * KP + e]) + red[3 * KP * KP + e];
    partials[(int64_t)e * gridDim.x + slot] = s;
  }
  __syncthreads();
}

// Fold per-lane column sums (column 16*cb + l%16) over lane groups and waves into partials (e = col).
template <int NB>
__device__ void fold_cols(double (&s)[NB], double* red, double* partials) {
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
  const int64_t slot = dev::xcd_slot(blockIdx.x, gridDim.x);
  if (threadIdx.x < KP) {
    const int e = threadIdx.x;
    partials[(int64_t)e * gridDim.x + slot] = ((red[e] + red[KP + e]) + red[2 * KP + e]) + red[3 * KP + e];
  }
  __syncthreads();
}

// B-operand fragments of a k x k matrix M (row-major, FP64): frag[kb][cb] = M[4kb + l/16][16cb + l%16].
template <int NB>
__device__ __forceinline__ void load_bfrag(const double* M, int k, double scale, double (&frag)[4 * NB][NB]) {
  const int l = threadIdx.x & 63, g = l >> 4, c = l & 15;
#pragma unroll
  for (int kb = 0; kb < 4 * NB; ++kb)
#pragma unroll
    for (int cb = 0; cb < NB; ++cb) {
      const int r = 4 * kb + g, col = 16 * cb + c;
      frag[kb][cb] = (M && r < k && col < k) ? scale * M[r * k + col] : 0.0;
    }
}

// ----------------------------------------------------------------------------- Gram X^T Y

template <typename T, int NB>
__global__ __launch_bounds__(256) void mf_gram_kernel(int64_t N, int k, const T* __restrict__ X, int ldx,
                                                      const T* __restrict__ Y, int ldy, double* partials) {
  __shared__ __align__(16) double red[4 * 16 * NB * 16 * NB];
  const int l = threadIdx.x & 63, g = l >> 4, c = l & 15;
  d4 acc[NB][NB];
#pragma unroll
  for (int i = 0; i < NB; ++i)
#pragma unroll
    for (int j = 0; j < NB; ++j) acc[i][j] = zero4();
  const WaveRange wr = wave_range((N + 3) / 4);
  for (int64_t q = wr.begin; q < wr.end; ++q) {
    const int64_t r = 4 * q + g;
    double x[NB], y[NB];
#pragma unroll
    for (int cb = 0; cb < NB; ++cb) {
      const int col = 16 * cb + c;
      const bool ok = r < N && col < k;
      x[cb] = ldz(X + r * ldx + col, ok);
      y[cb] = ldz(Y + r * ldy + col, ok);
    }
#pragma unroll
    for (int ia = 0; ia < NB; ++ia)
#pragma unroll
      for (int jb = 0; jb < NB; ++jb) acc[ia][jb] = mfma(x[ia], y[jb], acc[ia][jb]);
  }
  fold_kxk<NB>(acc, red, partials);
}

// ----------------------------------------------------------------------------- SpMM + Gram

template <typename T>
struct SpmmGramArgs {
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
  double* partials;
};

// Q = alpha P + beta K P (arithmetic in T) and G = P^T Q (FP64, MFMA).  One row per lane group of
// 16 lanes; lane l covers columns l%16 (+16).  The 16 lanes of a row share each matrix entry.
template <typename T, int NB, bool SELL>
__global__ __launch_bounds__(256) void mf_spmm_gram_kernel(SpmmGramArgs<T> a) {
  __shared__ __align__(16) double red[4 * 16 * NB * 16 * NB];
  const int l = threadIdx.x & 63, g = l >> 4, c = l & 15;
  d4 acc[NB][NB];
#pragma unroll
  for (int i = 0; i < NB; ++i)
#pragma unroll
    for (int j = 0; j < NB; ++j) acc[i][j] = zero4();
  const WaveRange wr = wave_range((a.N + 3) / 4);
  constexpr int U = 8;
  for (int64_t q = wr.begin; q < wr.end; ++q) {
    const int64_t r = 4 * q + g;
    const bool rok = r < a.N;
    T s[NB];
#pragma unroll
    for (int cb = 0; cb < NB; ++cb) s[cb] = T(0);
    int64_t base = 0, stride = 1, len = 0;
    if (rok) {
      if constexpr (SELL) {
        const int64_t sl = r / a.C;
        base = a.sptr[sl] + (r - sl * a.C);
        stride = a.C;
        len = a.sw[sl];
      } else {
        base = a.rowptr[r];
        len = a.rowptr[r + 1] - base;
      }
    }
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
#pragma unroll
      for (int cb = 0; cb < NB; ++cb) {
        const int col = 16 * cb + c;
        if (col < a.k) {
          T xv[U];
#pragma unroll
          for (int u = 0; u < U; ++u) xv[u] = a.P[(int64_t)ci[u] * a.k + col];
#pragma unroll
          for (int u = 0; u < U; ++u) s[cb] = fma(v[u], xv[u], s[cb]);
        }
      }
    }
    double p[NB], qv[NB];
#pragma unroll
    for (int cb = 0; cb < NB; ++cb) {
      const int col = 16 * cb + c;
      const bool ok = rok && col < a.k;
      const T pv = ok ? a.P[r * a.k + col] : T(0);
      const T out = (T)a.beta * s[cb] + (T)a.alpha * pv;
      if (ok) a.Q[r * a.k + col] = out;
      p[cb] = ok ? (double)pv : 0.0;
      qv[cb] = ok ? (double)out : 0.0;
    }
#pragma unroll
    for (int ia = 0; ia < NB; ++ia)
#pragma unroll
      for (int jb = 0; jb < NB; ++jb) acc[ia][jb] = mfma(p[ia], qv[jb], acc[ia][jb]);
  }
  fold_kxk<NB>(acc, red, a.partials);
}

// ----------------------------------------------------------------------------- tile helpers

// Load a 16-row tile of a row-major block (ld = k) into D layout regs d[cb][v] (row 4v + g, col
// 16cb + c) and, when `lds` is given, into the wave's LDS copy.
template <typename T, int NB>
__device__ __forceinline__ void load_tile(const T* M, int64_t N, int k, int64_t row0, double (&d)[NB][4],
                                          double* lds) {
  const int l = threadIdx.x & 63, g = l >> 4, c = l & 15;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int rr = 4 * v + g;
    const int64_t r = row0 + rr;
#pragma unroll
    for (int cb = 0; cb < NB; ++cb) {
      const int col = 16 * cb + c;
      d[cb][v] = ldz(M + r * k + col, r < N && col < k);
      if (lds) lds[rr * MGeom<NB>::LDT + col] = d[cb][v];
    }
  }
}

// A-operand fragments of the wave's LDS tile: a[kb] = tile[l % 16][4kb + l/16].
template <int NB>
__device__ __forceinline__ void read_afrag(const double* lds, double (&a)[4 * NB]) {
  const int l = threadIdx.x & 63;
#pragma unroll
  for (int kb = 0; kb < 4 * NB; ++kb) a[kb] = lds[(l & 15) * MGeom<NB>::LDT + 4 * kb + (l >> 4)];
}

// D = C + A_tile * M  for every column block (C given in D layout).
template <int NB>
__device__ __forceinline__ void tile_rmul(const double (&a)[4 * NB], const double (&bf)[4 * NB][NB],
                                          const double (&cin)[NB][4], d4 (&out)[NB]) {
#pragma unroll
  for (int cb = 0; cb < NB; ++cb) {
    d4 acc = d4{cin[cb][0], cin[cb][1], cin[cb][2], cin[cb][3]};
#pragma unroll
    for (int kb = 0; kb < 4 * NB; ++kb) acc = mfma(a[kb], bf[kb][cb], acc);
    out[cb] = acc;
  }
}

template <typename T, int NB>
__device__ __forceinline__ void store_tile(T* M, int64_t N, int k, int64_t row0, const d4 (&d)[NB]) {
  const int l = threadIdx.x & 63, g = l >> 4, c = l & 15;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int64_t r = row0 + 4 * v + g;
#pragma unroll
    for (int cb = 0; cb < NB; ++cb) {
      const int col = 16 * cb + c;
      if (r < N && col < k) M[r * k + col] = (T)d[cb][v];
    }
  }
}

__device__ __forceinline__ double dinv_row(const double* dinv, int64_t r, int64_t N) {
  return (dinv && r < N) ? dinv[r] : 1.0;
}

// ----------------------------------------------------------------------------- block CG update

struct CgUpdArgs {
  int64_t N;
  int k;
  void* X;
  const void* P;
  void* R;
  const void* Q;
  const double* alpha;
  const double* dinv;  // inverse Jacobi diagonal, or null for no preconditioning
  double *pg, *pt, *pn;
};

// X += P alpha; R -= Q alpha; Z = D^-1 R; gamma = R^T Z; T = Q^T Z; nrm = diag(R^T R)
template <typename T, int NB>
__global__ __launch_bounds__(256) void mf_cg_update_kernel(CgUpdArgs a) {
  using MG = MGeom<NB>;
  constexpr int KP = MG::KP;
  constexpr int LDSN = (8 * MG::TILE > 4 * KP * KP) ? 8 * MG::TILE : 4 * KP * KP;
  __shared__ __align__(16) double lds[LDSN];
  const int l = threadIdx.x & 63, w = threadIdx.x >> 6, g = l >> 4;
  double* Pl = lds + (2 * w) * MG::TILE;
  double* Ql = Pl + MG::TILE;
  const T* P = static_cast<const T*>(a.P);
  const T* Q = static_cast<const T*>(a.Q);
  T* X = static_cast<T*>(a.X);
  T* R = static_cast<T*>(a.R);
  double af[4 * NB][NB], naf[4 * NB][NB];
  load_bfrag<NB>(a.alpha, a.k, 1.0, af);
  load_bfrag<NB>(a.alpha, a.k, -1.0, naf);
  d4 gam[NB][NB], tac[NB][NB];
  double nrm[NB];
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    nrm[i] = 0.0;
#pragma unroll
    for (int j = 0; j < NB; ++j) gam[i][j] = tac[i][j] = zero4();
  }
  const WaveRange wr = wave_range((a.N + 15) / 16);
  for (int64_t t = wr.begin; t < wr.end; ++t) {
    const int64_t row0 = 16 * t;
    double pd[NB][4], qd[NB][4], xd[NB][4], rd[NB][4];
    load_tile<T, NB>(P, a.N, a.k, row0, pd, Pl);
    load_tile<T, NB>(Q, a.N, a.k, row0, qd, Ql);
    load_tile<T, NB>(X, a.N, a.k, row0, xd, nullptr);
    load_tile<T, NB>(R, a.N, a.k, row0, rd, nullptr);
    double dv[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) dv[v] = dinv_row(a.dinv, row0 + 4 * v + g, a.N);
    __builtin_amdgcn_wave_barrier();
    double pa[4 * NB], qa[4 * NB];
    read_afrag<NB>(Pl, pa);
    read_afrag<NB>(Ql, qa);
    d4 xn[NB], rn[NB];
    tile_rmul<NB>(pa, af, xd, xn);
    tile_rmul<NB>(qa, naf, rd, rn);
    store_tile<T, NB>(X, a.N, a.k, row0, xn);
    store_tile<T, NB>(R, a.N, a.k, row0, rn);
    double z[NB][4], rr[NB][4];
#pragma unroll
    for (int cb = 0; cb < NB; ++cb)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        // stored values are rounded to T; use the rounded ones so that FP32 runs see what memory holds
        rr[cb][v] = (double)(T)rn[cb][v];
        z[cb][v] = rr[cb][v] * dv[v];
        nrm[cb] = fma(rr[cb][v], rr[cb][v], nrm[cb]);
      }
#pragma unroll
    for (int v = 0; v < 4; ++v)
#pragma unroll
      for (int ia = 0; ia < NB; ++ia)
#pragma unroll
        for (int jb = 0; jb < NB; ++jb) {
          gam[ia][jb] = mfma(rr[ia][v], z[jb][v], gam[ia][jb]);
          tac[ia][jb] = mfma(qd[ia][v], z[jb][v], tac[ia][jb]);
        }
    __builtin_amdgcn_wave_barrier();
  }
  fold_kxk<NB>(gam, lds, a.pg);
  fold_kxk<NB>(tac, lds, a.pt);
  fold_cols<NB>(nrm, lds, a.pn);
}

// P = D^-1 R + P beta   (beta == nullptr: P = D^-1 R)
template <typename T, int NB>
__global__ __launch_bounds__(256) void mf_cg_pupdate_kernel(int64_t N, int k, T* __restrict__ P,
                                                            const T* __restrict__ R, const double* beta,
                                                            const double* dinv) {
  using MG = MGeom<NB>;
  __shared__ __align__(16) double lds[4 * MG::TILE];
  const int l = threadIdx.x & 63, w = threadIdx.x >> 6, g = l >> 4;
  double* Pl = lds + w * MG::TILE;
  double bf[4 * NB][NB];
  load_bfrag<NB>(beta, k, 1.0, bf);
  const WaveRange wr = wave_range((N + 15) / 16);
  for (int64_t t = wr.begin; t < wr.end; ++t) {
    const int64_t row0 = 16 * t;
    double pd[NB][4], zd[NB][4];
    load_tile<T, NB>(P, N, k, row0, pd, Pl);
    load_tile<T, NB>(R, N, k, row0, zd, nullptr);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const double dv = dinv_row(dinv, row0 + 4 * v + g, N);
#pragma unroll
      for (int cb = 0; cb < NB; ++cb) zd[cb][v] *= dv;
    }
    __builtin_amdgcn_wave_barrier();
    d4 pn[NB];
    if (beta) {
      double pa[4 * NB];
      read_afrag<NB>(Pl, pa);
      tile_rmul<NB>(pa, bf, zd, pn);
    } else {
#pragma unroll
      for (int cb = 0; cb < NB; ++cb) pn[cb] = d4{zd[cb][0], zd[cb][1], zd[cb][2], zd[cb][3]};
    }
    store_tile<T, NB>(P, N, k, row0, pn);
    __builtin_amdgcn_wave_barrier();
  }
}

// Y = c0 Y + c1 X C   (contiguous blocks, ld = k)
template <typename T, int NB>
__global__ __launch_bounds__(256) void mf_rmul_kernel(int64_t N, int k, const T* __restrict__ X, const double* C,
                                                      double c0, double c1, T* Y) {
  using MG = MGeom<NB>;
  __shared__ __align__(16) double lds[4 * MG::TILE];
  const int w = threadIdx.x >> 6;
  double* Xl = lds + w * MG::TILE;
  double bf[4 * NB][NB];
  load_bfrag<NB>(C, k, c1, bf);
  const WaveRange wr = wave_range((N + 15) / 16);
  for (int64_t t = wr.begin; t < wr.end; ++t) {
    const int64_t row0 = 16 * t;
    double xd[NB][4], yd[NB][4];
    load_tile<T, NB>(X, N, k, row0, xd, Xl);
    if (c0 != 0.0) {
      load_tile<T, NB>(Y, N, k, row0, yd, nullptr);
#pragma unroll
      for (int cb = 0; cb < NB; ++cb)
#pragma unroll
        for (int v = 0; v < 4; ++v) yd[cb][v] *= c0;
    } else {
#pragma unroll
      for (int cb = 0; cb < NB; ++cb)
#pragma unroll
        for (int v = 0; v < 4; ++v) yd[cb][v] = 0.0;
    }
    __builtin_amdgcn_wave_barrier();
    double xa[4 * NB];
    read_afrag<NB>(Xl, xa);
    d4 yn[NB];
    tile_rmul<NB>(xa, bf, yd, yn);
    store_tile<T, NB>(Y, N, k, row0, yn);
    __builtin_amdgcn_wave_barrier();
  }
}

// ----------------------------------------------------------------------------- block Gram-Schmidt
// Projection of W against nblk blocks V_i = V0 + i * vstride (block GMRES): G_i = V_i^T W for all i
// in one pass that reads W once, and W -= sum_i V_i C_i in one pass that reads and writes W once.
// MB blocks at most per launch (register budget: MB * NB^2 accumulators).

template <int NB>
constexpr int mgs_max_blocks() { return NB == 1 ? 4 : 2; }

template <typename T, int NB>
__global__ __launch_bounds__(256) void mf_mgram_kernel(int64_t N, int k, int nblk, const T* __restrict__ V0,
                                                       int64_t vstride, const T* __restrict__ W,
                                                       double* partials) {
  constexpr int MB = mgs_max_blocks<NB>();
  constexpr int KP = 16 * NB;
  __shared__ __align__(16) double red[4 * KP * KP];
  const int l = threadIdx.x & 63, g = l >> 4, c = l & 15;
  d4 acc[MB][NB][NB];
#pragma unroll
  for (int b = 0; b < MB; ++b)
#pragma unroll
    for (int i = 0; i < NB; ++i)
#pragma unroll
      for (int j = 0; j < NB; ++j) acc[b][i][j] = zero4();
  const WaveRange wr = wave_range((N + 3) / 4);
  // Every load of a step precedes its first matrix-core instruction. Rows past N and columns past k
  // are read at a valid element and multiplied by zero, so no load sits behind a branch.
  if constexpr (sizeof(T) == 4) {
    // FP32 blocks: FP32 matrix-core sums over one 16-row tile (4 quads), added in FP64 across tiles;
    // the FP64 accumulators keep the FP32 D layout.
    for (int64_t t = wr.begin; t < wr.end; t += 4) {
      float y[4][NB], x[4][MB][NB];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int64_t r = 4 * (t + u) + g;
        const bool rok = t + u < wr.end && r < N;
        const int64_t rr = rok ? r : (4 * t + g < N ? 4 * t + g : N - 1);
#pragma unroll
        for (int cb = 0; cb < NB; ++cb) {
          const int col = 16 * cb + c;
          const int cc = col < k ? col : k - 1;
          const float m = (rok && col < k) ? 1.0f : 0.0f;
          y[u][cb] = m * static_cast<float>(W[rr * k + cc]);
#pragma unroll
          for (int b = 0; b < MB; ++b)
            x[u][b][cb] = (b < nblk) ? m * static_cast<float>(V0[b * vstride + rr * k + cc]) : 0.0f;
        }
      }
#pragma unroll
      for (int b = 0; b < MB; ++b)
        if (b < nblk) {
#pragma unroll
          for (int ia = 0; ia < NB; ++ia)
#pragma unroll
            for (int jb = 0; jb < NB; ++jb) {
              f4m p = f4m{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
              for (int u = 0; u < 4; ++u) p = mfma32(x[u][b][ia], y[u][jb], p);
#pragma unroll
              for (int v = 0; v < 4; ++v) acc[b][ia][jb][v] += static_cast<double>(p[v]);
            }
        }
    }
  } else {
    constexpr int U = 2;  // quads per step
    for (int64_t q0 = wr.begin; q0 < wr.end; q0 += U) {
      double y[U][NB], x[U][MB][NB];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t r = 4 * (q0 + u) + g;
        const bool rok = q0 + u < wr.end && r < N;
        const int64_t rr = rok ? r : (4 * q0 + g < N ? 4 * q0 + g : N - 1);
#pragma unroll
        for (int cb = 0; cb < NB; ++cb) {
          const int col = 16 * cb + c;
          const int cc = col < k ? col : k - 1;
          const double m = (rok && col < k) ? 1.0 : 0.0;
          y[u][cb] = m * static_cast<double>(W[rr * k + cc]);
#pragma unroll
          for (int b = 0; b < MB; ++b)
            x[u][b][cb] = (b < nblk) ? m * static_cast<double>(V0[b * vstride + rr * k + cc]) : 0.0;
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int b = 0; b < MB; ++b)
          if (b < nblk) {
#pragma unroll
            for (int ia = 0; ia < NB; ++ia)
#pragma unroll
              for (int jb = 0; jb < NB; ++jb) acc[b][ia][jb] = mfma(x[u][b][ia], y[u][jb], acc[b][ia][jb]);
          }
    }
  }
#pragma unroll
  for (int b = 0; b < MB; ++b)
    if (b < nblk) {
      if constexpr (sizeof(T) == 4)
        fold_kxk32<NB>(acc[b], red, partials + (int64_t)b * KP * KP * gridDim.x);
      else
        fold_kxk<NB>(acc[b], red, partials + (int64_t)b * KP * KP * gridDim.x);
    }
}

// W -= sum_b V_b C_b, C_b = C + b * k * k (row-major k x k, FP64).  The coefficient blocks are
// staged once per workgroup in LDS (negated, zero padded); the A operand of each basis tile is read
// straight from device memory in the transposed order it needs (lane l: row l % 16, columns
// 4kb + l / 16, all within the tile's contiguous rows), and all basis tiles of a W tile are loaded
// before the first matrix-core instruction.
template <typename T, int NB>
__global__ __launch_bounds__(256) void mf_mrmul_kernel(int64_t N, int k, int nblk, const T* __restrict__ V0,
                                                       int64_t vstride, const double* C, T* W) {
  constexpr int MB = mgs_max_blocks<NB>();
  constexpr int KP = 16 * NB;
  __shared__ double Cs[MB * KP * KP];
  for (int e = threadIdx.x; e < MB * KP * KP; e += 256) {
    const int b = e / (KP * KP), rc = e % (KP * KP), r = rc / KP, c = rc % KP;
    Cs[e] = (b < nblk && r < k && c < k) ? -C[(int64_t)b * k * k + r * k + c] : 0.0;
  }
  __syncthreads();
  const int l = threadIdx.x & 63, g = l >> 4, c = l & 15;
  const WaveRange wr = wave_range((N + 15) / 16);
  for (int64_t t = wr.begin; t < wr.end; ++t) {
    const int64_t row0 = 16 * t;
    double yd[NB][4];
    load_tile<T, NB>(W, N, k, row0, yd, nullptr);
    double xa[MB][4 * NB];
    const int64_t ra = row0 + (l & 15);
#pragma unroll
    for (int b = 0; b < MB; ++b)
#pragma unroll
      for (int kb = 0; kb < 4 * NB; ++kb) {
        const int col = 4 * kb + (l >> 4);
        xa[b][kb] = (b < nblk) ? ldz(V0 + b * vstride + ra * k + col, ra < N && col < k) : 0.0;
      }
#pragma unroll
    for (int b = 0; b < MB; ++b) {
      if (b < nblk) {
        double bf[4 * NB][NB];
#pragma unroll
        for (int kb = 0; kb < 4 * NB; ++kb)
#pragma unroll
          for (int cb = 0; cb < NB; ++cb) bf[kb][cb] = Cs[b * KP * KP + (4 * kb + g) * KP + 16 * cb + c];
        d4 yn[NB];
        tile_rmul<NB>(xa[b], bf, yd, yn);
#pragma unroll
        for (int cb = 0; cb < NB; ++cb)
#pragma unroll
          for (int v = 0; v < 4; ++v) yd[cb][v] = yn[cb][v];
      }
    }
    d4 out[NB];
#pragma unroll
    for (int cb = 0; cb < NB; ++cb) out[cb] = d4{yd[cb][0], yd[cb][1], yd[cb][2], yd[cb][3]};
    store_tile<T, NB>(W, N, k, row0, out);
  }
}

// Single-column blocks (k = 1): the projection of w against nblk <= kMdotMax vectors is nblk dot
// products in one pass over w, and w -= sum_b c_b v_b one pass that reads and writes w once.
constexpr int kMdotMax = 16;

template <typename T>
__global__ __launch_bounds__(256) void mdot_kernel(int64_t n, int nblk, const T* __restrict__ V0, int64_t vstride,
                                                   const T* __restrict__ W, double* partials) {
  __shared__ double red[4 * kMdotMax];
  double acc[kMdotMax];
#pragma unroll
  for (int b = 0; b < kMdotMax; ++b) acc[b] = 0.0;
  const int64_t slot = dev::xcd_slot(blockIdx.x, gridDim.x);
  const int64_t per = (n + gridDim.x - 1) / gridDim.x;
  const int64_t lo = slot * per, hi = lo + per < n ? lo + per : n;
  for (int64_t i = lo + threadIdx.x; i < hi; i += 256) {
    const double w = (double)W[i];
#pragma unroll
    for (int b = 0; b < kMdotMax; ++b)
      if (b < nblk) acc[b] = fma((double)V0[b * vstride + i], w, acc[b]);
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int b = 0; b < kMdotMax; ++b) {
    double v = acc[b];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    if (lane == 0) red[wv * kMdotMax + b] = v;
  }
  __syncthreads();
  if (threadIdx.x < nblk) {
    const int b = threadIdx.x;
    partials[(int64_t)b * gridDim.x + slot] =
        ((red[b] + red[kMdotMax + b]) + red[2 * kMdotMax + b]) + red[3 * kMdotMax + b];
  }
}

template <typename T>
__global__ __launch_bounds__(256) void maxpy_kernel(int64_t n, int nblk, const T* __restrict__ V0, int64_t vstride,
                                                    const double* __restrict__ C, T* __restrict__ W) {
  __shared__ double cs[kMdotMax];
  if (threadIdx.x < nblk) cs[threadIdx.x] = C[threadIdx.x];
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  double w = (double)W[i];
#pragma unroll
  for (int b = 0; b < kMdotMax; ++b)
    if (b < nblk) w = fma(-cs[b], (double)V0[b * vstride + i], w);
  W[i] = (T)w;
}

// One workgroup per entry (b, a, c) of the nblk projection blocks: sum the slots in a fixed order,
// store C_b[a][c] and add it into the block Hessenberg matrix H (column-major, ldh) at row
// r0 + b k + a, column c0 + c.
__global__ __launch_bounds__(256) void mgs_finalize_kernel(const double* partials, int64_t nslots, int k, int KP,
                                                           double* C, double* H, int ldh, int r0, int c0,
                                                           int accumulate) {
  __shared__ double sred[256];
  const int idx = blockIdx.x;
  const int b = idx / (k * k), a = (idx / k) % k, cc = idx % k;
  const double* p = partials + ((int64_t)b * KP * KP + (int64_t)a * KP + cc) * nslots;
  double acc = 0.0;
  for (int64_t j = threadIdx.x; j < nslots; j += 256) acc += p[j];
  sred[threadIdx.x] = acc;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) sred[threadIdx.x] += sred[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double v = sred[0];
    C[idx] = v;
    double* h = H + (int64_t)(c0 + cc) * ldh + r0 + b * k + a;
    *h = accumulate ? *h + v : v;
  }
}

// Persistent grid: the chip's resident capacity for the kernel, capped so that every wave owns at
// least ~4 work units.
int64_t mf_blocks(bkts_ctx ctx, const void* kernel, int64_t units) {
  const int64_t waves = (units + 3) / 4;
  int64_t nb = (waves + 3) / 4;
  const int64_t cap = (int64_t)blocks_per_cu(kernel) * ctx->num_cu;
  if (nb > cap) nb = cap;
  return nb < 1 ? 1 : nb;
}

template <typename K>
int64_t mf_blocks(bkts_ctx ctx, K kernel, int64_t units) {
  return mf_blocks(ctx, reinterpret_cast<const void*>(kernel), units);
}

}  // namespace

bool mf_eligible(int k) { return k >= 8 && k <= 32; }

#define BKTS_NB_DISPATCH(k, CALL)            \
  do {                                       \
    if ((k) <= 16) { constexpr int NB = 1; CALL; } \
    else { constexpr int NB = 2; CALL; }     \
  } while (0)

void mf_gram(bkts_ctx ctx, int dtype, int64_t N, int k, const void* X, int ldx, const void* Y, int ldy, double* G) {
  const int KP = k <= 16 ? 16 : 32;
  const int64_t nb = mf_blocks(ctx, dtype == BKTS_F64 ? (k <= 16 ? (const void*)mf_gram_kernel<double, 1> : (const void*)mf_gram_kernel<double, 2>)
                                                     : (k <= 16 ? (const void*)mf_gram_kernel<float, 1> : (const void*)mf_gram_kernel<float, 2>),
                                (N + 3) / 4);
  double* part = ctx->ws.get<double>("mf_gram_part", (size_t)KP * KP * nb);
  ProfScope prof(ctx, BKTS_K_GRAM, 2.0 * N * k * esize(dtype));
  if (dtype == BKTS_F64)
    BKTS_NB_DISPATCH(k, launch(ctx, (mf_gram_kernel<double, NB>), dim3(nb), dim3(256), 0, N, k,
                                            static_cast<const double*>(X), ldx, static_cast<const double*>(Y), ldy,
                                            part));
  else
    BKTS_NB_DISPATCH(k, launch(ctx, (mf_gram_kernel<float, NB>), dim3(nb), dim3(256), 0, N, k,
                                            static_cast<const float*>(X), ldx, static_cast<const float*>(Y), ldy,
                                            part));
  BKTS_HIP(hipGetLastError());
  prof.end();
  finalize_gram(ctx, part, (int)nb, k, KP, G);
}

void mf_spmm_gram(bkts_ctx ctx, const bkts_op_s& op, int dtype, int k, double alpha, const void* P, double beta,
                  void* Q, double* G) {
  const int KP = k <= 16 ? 16 : 32;
  const int64_t N = op.N;
  const bool sell0 = op.format == BKTS_FMT_SELL;
  const void* kern =
      dtype == BKTS_F64
          ? (k <= 16 ? (sell0 ? (const void*)mf_spmm_gram_kernel<double, 1, true> : (const void*)mf_spmm_gram_kernel<double, 1, false>)
                     : (sell0 ? (const void*)mf_spmm_gram_kernel<double, 2, true> : (const void*)mf_spmm_gram_kernel<double, 2, false>))
          : (k <= 16 ? (sell0 ? (const void*)mf_spmm_gram_kernel<float, 1, true> : (const void*)mf_spmm_gram_kernel<float, 1, false>)
                     : (sell0 ? (const void*)mf_spmm_gram_kernel<float, 2, true> : (const void*)mf_spmm_gram_kernel<float, 2, false>));
  const int64_t nb = mf_blocks(ctx, kern, (N + 3) / 4);
  double* part = ctx->ws.get<double>("mf_sg_part", (size_t)KP * KP * nb);
  const bool sell = op.format == BKTS_FMT_SELL;
  const double sv = esize(dtype);
  ProfScope prof(ctx, BKTS_K_SPMM, op.nnz * (sv + 4.0) + 4.0 * (N + 1) + 2.0 * N * k * sv);
  auto go = [&](auto tag) {
    using T = decltype(tag);
    SpmmGramArgs<T> a{};
    a.N = N;
    a.k = k;
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
    a.partials = part;
    if (sell)
      BKTS_NB_DISPATCH(k, launch(ctx, (mf_spmm_gram_kernel<T, NB, true>), dim3(nb), dim3(256), 0,
                                              a));
    else
      BKTS_NB_DISPATCH(k, launch(ctx, (mf_spmm_gram_kernel<T, NB, false>), dim3(nb), dim3(256), 0,
                                              a));
  };
  if (dtype == BKTS_F64)
    go(double{});
  else
    go(float{});
  BKTS_HIP(hipGetLastError());
  prof.end();
  finalize_gram(ctx, part, (int)nb, k, KP, G);
}

void mf_cg_update(bkts_ctx ctx, int dtype, int64_t N, int k, void* X, const void* P, void* R, const void* Q,
                  const double* alpha, const double* dinv, double* gamma,
                  double* Tm, double* nrm) {
  const int KP = k <= 16 ? 16 : 32;
  const int64_t nb = mf_blocks(ctx, dtype == BKTS_F64 ? (k <= 16 ? (const void*)mf_cg_update_kernel<double, 1> : (const void*)mf_cg_update_kernel<double, 2>)
                                                     : (k <= 16 ? (const void*)mf_cg_update_kernel<float, 1> : (const void*)mf_cg_update_kernel<float, 2>),
                                (N + 15) / 16);
  const size_t np = (size_t)KP * KP * nb;
  double* pg = ctx->ws.get<double>("mf_cg_pg", np);
  double* pt = ctx->ws.get<double>("mf_cg_pt", np);
  double* pn = ctx->ws.get<double>("mf_cg_pn", (size_t)KP * nb);
  CgUpdArgs a{N, k, X, P, R, Q, alpha, dinv, pg, pt, pn};
  ProfScope prof(ctx, BKTS_K_CG_UPDATE, 6.0 * N * k * esize(dtype) + (dinv ? 8.0 * N : 0.0));
  if (dtype == BKTS_F64)
    BKTS_NB_DISPATCH(k, launch(ctx, (mf_cg_update_kernel<double, NB>), dim3(nb), dim3(256), 0, a));
  else
    BKTS_NB_DISPATCH(k, launch(ctx, (mf_cg_update_kernel<float, NB>), dim3(nb), dim3(256), 0, a));
  BKTS_HIP(hipGetLastError());
  prof.end();
  const FoldSet sets[3] = {{pg, KP, 0, gamma}, {pt, KP, 0, Tm}, {pn, KP, 1, nrm}};
  finalize_sets(ctx, (int)nb, k, sets, 3);
}

void mf_cg_pupdate(bkts_ctx ctx, int dtype, int64_t N, int k, void* P, const void* R, const double* beta,
                   const double* dinv) {
  const int64_t nb = mf_blocks(ctx, dtype == BKTS_F64 ? (k <= 16 ? (const void*)mf_cg_pupdate_kernel<double, 1> : (const void*)mf_cg_pupdate_kernel<double, 2>)
                                                     : (k <= 16 ? (const void*)mf_cg_pupdate_kernel<float, 1> : (const void*)mf_cg_pupdate_kernel<float, 2>),
                                (N + 15) / 16);
  ProfScope prof(ctx, BKTS_K_CG_PUPDATE, (beta ? 3.0 : 2.0) * N * k * esize(dtype) + (dinv ? 8.0 * N : 0.0));
  if (dtype == BKTS_F64)
    BKTS_NB_DISPATCH(k, launch(ctx, (mf_cg_pupdate_kernel<double, NB>), dim3(nb), dim3(256), 0, N, k, static_cast<double*>(P), static_cast<const double*>(R), beta, dinv));
  else
    BKTS_NB_DISPATCH(k, launch(ctx, (mf_cg_pupdate_kernel<float, NB>), dim3(nb), dim3(256), 0, N, k, static_cast<float*>(P), static_cast<const float*>(R), beta, dinv));
  BKTS_HIP(hipGetLastError());
}

void mf_rmul(bkts_ctx ctx, int dtype, int64_t N, int k, const void* X, const double* C, double c0, double c1,
             void* Y) {
  const int64_t nb = mf_blocks(ctx, dtype == BKTS_F64 ? (k <= 16 ? (const void*)mf_rmul_kernel<double, 1> : (const void*)mf_rmul_kernel<double, 2>)
                                                     : (k <= 16 ? (const void*)mf_rmul_kernel<float, 1> : (const void*)mf_rmul_kernel<float, 2>),
                                (N + 15) / 16);
  ProfScope prof(ctx, BKTS_K_OTHER, (c0 != 0.0 ? 3.0 : 2.0) * N * k * esize(dtype));
  if (dtype == BKTS_F64)
    BKTS_NB_DISPATCH(k, launch(ctx, (mf_rmul_kernel<double, NB>), dim3(nb), dim3(256), 0, N, k,
                                            static_cast<const double*>(X), C, c0, c1, static_cast<double*>(Y)));
  else
    BKTS_NB_DISPATCH(k, launch(ctx, (mf_rmul_kernel<float, NB>), dim3(nb), dim3(256), 0, N, k,
                                            static_cast<const float*>(X), C, c0, c1, static_cast<float*>(Y)));
  BKTS_HIP(hipGetLastError());
}

int mf_mgs_max_blocks(int k) { return k <= 16 ? mgs_max_blocks<1>() : mgs_max_blocks<2>(); }

void mf_mgram(bkts_ctx ctx, int dtype, int64_t N, int k, int nblk, const void* V0, int64_t vstride, const void* W,
              double* partials_out, int* nslots_out) {
  const int64_t nb = mf_blocks(ctx, dtype == BKTS_F64 ? (k <= 16 ? (const void*)mf_mgram_kernel<double, 1> : (const void*)mf_mgram_kernel<double, 2>)
                                                     : (k <= 16 ? (const void*)mf_mgram_kernel<float, 1> : (const void*)mf_mgram_kernel<float, 2>),
                                (N + 3) / 4);
  BKTS_REQUIRE(nblk >= 1 && nblk <= mf_mgs_max_blocks(k), "mf_mgram: bad block count %d", nblk);
  ProfScope prof(ctx, BKTS_K_GRAM, (1.0 + nblk) * N * k * esize(dtype));
  if (dtype == BKTS_F64)
    BKTS_NB_DISPATCH(k, launch(ctx, (mf_mgram_kernel<double, NB>), dim3(nb), dim3(256), 0, N, k, nblk,
                               static_cast<const double*>(V0), vstride, static_cast<const double*>(W), partials_out));
  else
    BKTS_NB_DISPATCH(k, launch(ctx, (mf_mgram_kernel<float, NB>), dim3(nb), dim3(256), 0, N, k, nblk,
                               static_cast<const float*>(V0), vstride, static_cast<const float*>(W), partials_out));
  BKTS_HIP(hipGetLastError());
  *nslots_out = (int)nb;
}

int64_t mf_mgram_slots(bkts_ctx ctx, int dtype, int64_t N, int k) {
  return mf_blocks(ctx, dtype == BKTS_F64 ? (k <= 16 ? (const void*)mf_mgram_kernel<double, 1> : (const void*)mf_mgram_kernel<double, 2>)
                                         : (k <= 16 ? (const void*)mf_mgram_kernel<float, 1> : (const void*)mf_mgram_kernel<float, 2>),
                   (N + 3) / 4);
}

void mf_mrmul(bkts_ctx ctx, int dtype, int64_t N, int k, int nblk, const void* V0, int64_t vstride, const double* C,
              void* W) {
  const int64_t nb = mf_blocks(ctx, dtype == BKTS_F64 ? (k <= 16 ? (const void*)mf_mrmul_kernel<double, 1> : (const void*)mf_mrmul_kernel<double, 2>)
                                                     : (k <= 16 ? (const void*)mf_mrmul_kernel<float, 1> : (const void*)mf_mrmul_kernel<float, 2>),
                                (N + 15) / 16);
  BKTS_REQUIRE(nblk >= 1 && nblk <= mf_mgs_max_blocks(k), "mf_mrmul: bad block count %d", nblk);
  ProfScope prof(ctx, BKTS_K_OTHER, (2.0 + nblk) * N * k * esize(dtype));
  if (dtype == BKTS_F64)
    BKTS_NB_DISPATCH(k, launch(ctx, (mf_mrmul_kernel<double, NB>), dim3(nb), dim3(256), 0, N, k, nblk,
                               static_cast<const double*>(V0), vstride, C, static_cast<double*>(W)));
  else
    BKTS_NB_DISPATCH(k, launch(ctx, (mf_mrmul_kernel<float, NB>), dim3(nb), dim3(256), 0, N, k, nblk,
                               static_cast<const float*>(V0), vstride, C, static_cast<float*>(W)));
  BKTS_HIP(hipGetLastError());
}

void mf_mgs_finalize(bkts_ctx ctx, const double* partials, int nslots, int k, int nblk, double* C, double* H, int ldh,
                     int r0, int c0, bool accumulate) {
  const int KP = k == 1 ? 1 : k <= 16 ? 16 : 32;
  ProfScope prof(ctx, BKTS_K_SMALL, 8.0 * nblk * KP * KP * nslots);
  launch(ctx, mgs_finalize_kernel, dim3(nblk * k * k), dim3(256), 0, partials, (int64_t)nslots, k, KP, C, H, ldh, r0,
         c0, accumulate ? 1 : 0);
  BKTS_HIP(hipGetLastError());
}

int mdot_max_blocks() { return kMdotMax; }

int64_t mdot_slots(bkts_ctx ctx, int64_t n) {
  const int64_t cap = 4 * (int64_t)ctx->num_cu;
  const int64_t want = (n + 4095) / 4096;
  return std::max<int64_t>(1, std::min(cap, want));
}

void mdot(bkts_ctx ctx, int dtype, int64_t n, int nblk, const void* V0, int64_t vstride, const void* W,
          double* partials_out, int* nslots_out) {
  BKTS_REQUIRE(nblk >= 1 && nblk <= kMdotMax, "mdot: bad block count %d", nblk);
  const int64_t ns = mdot_slots(ctx, n);
  ProfScope prof(ctx, BKTS_K_GRAM, (1.0 + nblk) * n * esize(dtype));
  if (dtype == BKTS_F64)
    launch(ctx, mdot_kernel<double>, dim3(ns), dim3(256), 0, n, nblk, static_cast<const double*>(V0), vstride,
           static_cast<const double*>(W), partials_out);
  else
    launch(ctx, mdot_kernel<float>, dim3(ns), dim3(256), 0, n, nblk, static_cast<const float*>(V0), vstride,
           static_cast<const float*>(W), partials_out);
  BKTS_HIP(hipGetLastError());
  *nslots_out = (int)ns;
}

void maxpy(bkts_ctx ctx, int dtype, int64_t n, int nblk, const void* V0, int64_t vstride, const double* C, void* W) {
  BKTS_REQUIRE(nblk >= 1 && nblk <= kMdotMax, "maxpy: bad block count %d", nblk);
  ProfScope prof(ctx, BKTS_K_OTHER, (2.0 + nblk) * n * esize(dtype));
  const dim3 grid((unsigned)((n + 255) / 256));
  if (dtype == BKTS_F64)
    launch(ctx, maxpy_kernel<double>, grid, dim3(256), 0, n, nblk, static_cast<const double*>(V0), vstride, C,
           static_cast<double*>(W));
  else
    launch(ctx, maxpy_kernel<float>, grid, dim3(256), 0, n, nblk, static_cast<const float*>(V0), vstride, C,
           static_cast<float*>(W));
  BKTS_HIP(hipGetLastError());
}

}  // namespace bkts

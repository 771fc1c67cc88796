// Deflating solve of a k x k Gram system on one workgroup, shared by the block-CG solver and the
// grouped serving kernels.
#pragma once

#include "devcommon.hpp"
#include "../../include/bkts.h"

namespace bkts {
namespace dev {

constexpr int KM = BKTS_MAX_K;
constexpr int kSolveThreads = 256;

template <int KMAX>
struct SolveLdsT {
  double M[KMAX][2 * KMAX + 1];  // augmented [G | S], Jacobi scaled
  double d[KMAX];
  int active[KMAX];
};
using SolveLds = SolveLdsT<KM>;

// out = sign * G^+ S for k x k row-major G, S in device memory, run by all kSolveThreads threads
// of the block.  G^+ inverts the symmetric part of G on the directions that survive symmetric
// elimination of the Jacobi-scaled matrix D G D (D = diag(G)^-1/2, unit diagonal) in index order:
// a pivot (the Schur-complement diagonal, i.e. the squared Cholesky pivot) below `eps` marks its
// direction as numerically dependent on the earlier ones, and that row and column are dropped
// (the corresponding rows of the result are zero).  Gauss-Jordan on [D G D | D S] keeps every
// step a parallel update of the whole augmented matrix, with two barriers per pivot.
template <int KMAX>
__device__ inline void spd_solve_dev_t(int k, const double* Gin, const double* S, double sign, double eps, double* out,
                                       int* ndefl, SolveLdsT<KMAX>& sm) {
  const int t = threadIdx.x;
  const int w2 = 2 * k;
  for (int e = t; e < k * k; e += kSolveThreads) {
    const int i = e / k, j = e % k;
    sm.M[i][j] = 0.5 * (Gin[i * k + j] + Gin[j * k + i]);
    sm.M[i][k + j] = S[i * k + j];
  }
  __syncthreads();
  if (t < k) {
    const double g = sm.M[t][t];
    const bool ok = g > 0.0 && isfinite(g);
    sm.d[t] = ok ? rsqrt(g) : 0.0;
    sm.active[t] = ok ? 1 : 0;
  }
  __syncthreads();
  for (int e = t; e < k * w2; e += kSolveThreads) {
    const int i = e / w2, c = e % w2;
    sm.M[i][c] *= c < k ? sm.d[i] * sm.d[c] : sm.d[i];
  }
  __syncthreads();
  constexpr int EPT = (KMAX * 2 * KMAX + kSolveThreads - 1) / kSolveThreads;  // elements per thread
  int ri[EPT], ci[EPT];  // this thread's elements of the augmented matrix (fixed for all pivots)
#pragma unroll
  for (int q = 0; q < EPT; ++q) {
    const int e = t + q * kSolveThreads;
    ri[q] = e < k * w2 ? e / w2 : -1;
    ci[q] = e < k * w2 ? e % w2 : 0;
  }
  for (int j = 0; j < k; ++j) {
    const double p = sm.M[j][j];
    const bool keep = sm.active[j] && p > eps;
    const double rp = keep ? 1.0 / p : 0.0;
    double nv[EPT];
#pragma unroll
    for (int q = 0; q < EPT; ++q) {
      const int i = ri[q], c = ci[q];
      nv[q] = 0.0;
      if (i >= 0) {
        const double mic = sm.M[i][c];
        if (!keep)
          nv[q] = (i == j || c == j) ? 0.0 : mic;
        else if (i == j)
          nv[q] = mic * rp;
        else
          nv[q] = mic - sm.M[i][j] * (sm.M[j][c] * rp);
      }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < EPT; ++q)
      if (ri[q] >= 0) sm.M[ri[q]][ci[q]] = nv[q];
    if (t == 0 && !keep) sm.active[j] = 0;
    __syncthreads();
  }
  for (int e = t; e < k * k; e += kSolveThreads) {
    const int i = e / k, c = e % k;
    out[e] = sm.active[i] ? sign * sm.d[i] * sm.M[i][k + c] : 0.0;
  }
  if (t == 0 && ndefl) {
    int nd = 0;
    for (int i = 0; i < k; ++i) nd += sm.active[i] ? 0 : 1;
    *ndefl = nd;
  }
  __syncthreads();
}

__device__ inline void spd_solve_dev(int k, const double* Gin, const double* S, double sign, double eps, double* out,
                                     int* ndefl, SolveLds& sm) {
  spd_solve_dev_t<KM>(k, Gin, S, sign, eps, out, ndefl, sm);
}

// Threads per entry for folding E partial entries with one 256-thread workgroup.
constexpr int fold_tpe(int E) {
  int g = 1;
  while (2 * g * E <= kSolveThreads && g < kSolveThreads) g *= 2;
  return g;
}

// out[e] = sum over s of partials[e * nslots + s] for e < E, in a fixed order (strided partial
// sums per thread, then a fixed tree); all kSolveThreads threads, `red` holds kSolveThreads doubles.
template <int E>
__device__ inline void fold_slots(const double* partials, int64_t nslots, double* out, double* red) {
  constexpr int G = fold_tpe(E);
  constexpr int EPP = kSolveThreads / G;
  const int t = threadIdx.x, j = t % G;
  for (int e0 = 0; e0 < E; e0 += EPP) {
    const int e = e0 + t / G;
    double acc = 0.0;
    if (e < E)
      for (int64_t s = j; s < nslots; s += G) acc += partials[(int64_t)e * nslots + s];
    red[t] = acc;
    __syncthreads();
    for (int off = G / 2; off > 0; off >>= 1) {
      if (j < off) red[t] += red[t + off];
      __syncthreads();
    }
    if (j == 0 && e < E) out[e] = red[t];
    __syncthreads();
  }
}

// True in the workgroup that finishes last among `expected` workgroups sharing a device-scope
// counter (which the caller resets).  Global writes made before the call by every one of them are
// visible to the last one.
__device__ inline bool last_of(unsigned* counter, unsigned expected) {
  __shared__ int last;
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) last = atomicAdd(counter, 1u) == expected - 1 ? 1 : 0;
  __syncthreads();
  if (last) __threadfence();
  return last != 0;
}

__device__ inline bool last_workgroup(unsigned* counter) { return last_of(counter, gridDim.x); }

}  // namespace dev
}  // namespace bkts

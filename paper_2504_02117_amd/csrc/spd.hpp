// Truncated (deflating) Cholesky solve of a k x k Gram system on one workgroup, shared by the
// block-CG solver and the grouped serving kernels.
#pragma once

#include "devcommon.hpp"
#include "../../include/bkts.h"

namespace bkts {
namespace dev {

constexpr int KM = BKTS_MAX_K;

struct SolveLds {
  double L[KM][KM + 1];
  double Y[KM][KM + 1];
  double sc[KM];
  int active[KM];
};

// out = sign * G^+ S for k x k row-major G, S (device or LDS), run by threads 0..63 of the block
// (the others pass the barriers).  G^+ inverts the symmetric part of G restricted to the
// directions that survive a Cholesky factorisation of the Jacobi-scaled matrix D^-1/2 G D^-1/2: a
// pivot below `eps` (relative; the scaled matrix has unit diagonal) marks its direction as
// numerically dependent on the earlier ones, and that row and column are dropped.
__device__ inline void spd_solve_dev(int k, const double* Gin, const double* S, double sign, double eps, double* out,
                              int* ndefl, SolveLds& sm) {
  const int t = threadIdx.x;
  for (int e = t; e < k * k; e += blockDim.x) {
    const int i = e / k, j = e % k;
    sm.L[i][j] = 0.5 * (Gin[i * k + j] + Gin[j * k + i]);
  }
  __syncthreads();
  if (t < k) {
    const double d = sm.L[t][t];
    const bool ok = d > 0.0 && isfinite(d);
    sm.sc[t] = ok ? rsqrt(d) : 0.0;
    sm.active[t] = ok ? 1 : 0;
  }
  __syncthreads();
  for (int e = t; e < k * k; e += blockDim.x) {
    const int i = e / k, j = e % k;
    sm.L[i][j] *= sm.sc[i] * sm.sc[j];
  }
  __syncthreads();
  for (int j = 0; j < k; ++j) {  // right-looking Cholesky of the lower triangle, with deflation
    if (t == 0) {
      const double p = sm.L[j][j];
      if (!sm.active[j] || !(p > eps)) {
        sm.active[j] = 0;
        sm.L[j][j] = 1.0;
      } else {
        sm.L[j][j] = sqrt(p);
      }
    }
    __syncthreads();
    const bool aj = sm.active[j];
    for (int i = j + 1 + t; i < k; i += blockDim.x) sm.L[i][j] = aj ? sm.L[i][j] / sm.L[j][j] : 0.0;
    __syncthreads();
    if (aj) {
      for (int e = t; e < k * k; e += blockDim.x) {
        const int i = e / k, l = e % k;
        if (i > j && l > j && l <= i) sm.L[i][l] -= sm.L[i][j] * sm.L[l][j];
      }
    }
    __syncthreads();
  }
  if (t < k) {  // solve (L L^T) y = D^-1/2 S[:, c] for the column c = t
    const int c = t;
    for (int i = 0; i < k; ++i) {
      double v = sm.active[i] ? sm.sc[i] * S[i * k + c] : 0.0;
      for (int l = 0; l < i; ++l) v -= sm.L[i][l] * sm.Y[l][c];
      sm.Y[i][c] = sm.active[i] ? v / sm.L[i][i] : 0.0;
    }
    for (int i = k - 1; i >= 0; --i) {
      double v = sm.Y[i][c];
      for (int l = i + 1; l < k; ++l) v -= sm.L[l][i] * sm.Y[l][c];
      sm.Y[i][c] = sm.active[i] ? v / sm.L[i][i] : 0.0;
    }
    for (int i = 0; i < k; ++i) out[i * k + c] = sign * sm.sc[i] * sm.Y[i][c];
  }
  if (t == 0 && ndefl) {
    int nd = 0;
    for (int i = 0; i < k; ++i) nd += sm.active[i] ? 0 : 1;
    *ndefl = nd;
  }
  __syncthreads();
}

}  // namespace dev
}  // namespace bkts

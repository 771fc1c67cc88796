// k x k dense kernels that run on one workgroup and keep every block-Krylov coefficient on the
// device in FP64: the truncated (deflating) Cholesky solve used by block CG, and helpers.
#include "devcommon.hpp"
#include "internal.hpp"

namespace bkts {
namespace {

constexpr int KM = BKTS_MAX_K;

// out = sign * G^+ S, where G^+ is the inverse of the symmetric part of G restricted to the
// directions that survive a Cholesky factorisation of the Jacobi-scaled matrix D^-1/2 G D^-1/2:
// a pivot below `eps` (relative, the scaled matrix has unit diagonal) marks its direction as
// numerically dependent on the earlier ones; that row and column are dropped (zero rows in out).
__global__ __launch_bounds__(64) void spd_solve_kernel(int k, const double* __restrict__ Gin,
                                                       const double* __restrict__ S, double sign, double eps,
                                                       double* __restrict__ out, int* ndefl) {
  __shared__ double L[KM][KM + 1];
  __shared__ double sc[KM];
  __shared__ int active[KM];
  __shared__ double Y[KM][KM + 1];
  const int t = threadIdx.x;
  for (int e = t; e < k * k; e += 64) {
    const int i = e / k, j = e % k;
    L[i][j] = 0.5 * (Gin[i * k + j] + Gin[j * k + i]);
  }
  __syncthreads();
  if (t < k) {
    const double d = L[t][t];
    const bool ok = d > 0.0 && isfinite(d);
    sc[t] = ok ? rsqrt(d) : 0.0;
    active[t] = ok ? 1 : 0;
  }
  __syncthreads();
  for (int e = t; e < k * k; e += 64) {
    const int i = e / k, j = e % k;
    L[i][j] *= sc[i] * sc[j];
  }
  __syncthreads();
  // right-looking Cholesky on the lower triangle with deflation
  for (int j = 0; j < k; ++j) {
    if (t == 0) {
      const double p = L[j][j];
      if (!active[j] || !(p > eps)) {
        active[j] = 0;
        L[j][j] = 1.0;
      } else {
        L[j][j] = sqrt(p);
      }
    }
    __syncthreads();
    const bool aj = active[j];
    for (int i = j + 1 + t; i < k; i += 64) L[i][j] = aj ? L[i][j] / L[j][j] : 0.0;
    __syncthreads();
    if (aj) {
      for (int e = t; e < k * k; e += 64) {
        const int i = e / k, l = e % k;
        if (i > j && l > j && l <= i) L[i][l] -= L[i][j] * L[l][j];
      }
    }
    __syncthreads();
  }
  // solve for every right-hand side column c (thread c): (L L^T) y = D^-1/2 S[:, c]
  if (t < k) {
    const int c = t;
    for (int i = 0; i < k; ++i) {
      double v = active[i] ? sc[i] * S[i * k + c] : 0.0;
      for (int l = 0; l < i; ++l) v -= L[i][l] * Y[l][c];
      Y[i][c] = active[i] ? v / L[i][i] : 0.0;
    }
    for (int i = k - 1; i >= 0; --i) {
      double v = Y[i][c];
      for (int l = i + 1; l < k; ++l) v -= L[l][i] * Y[l][c];
      Y[i][c] = active[i] ? v / L[i][i] : 0.0;
    }
    for (int i = 0; i < k; ++i) out[i * k + c] = sign * sc[i] * Y[i][c];
  }
  if (t == 0 && ndefl) {
    int nd = 0;
    for (int i = 0; i < k; ++i) nd += active[i] ? 0 : 1;
    *ndefl = nd;
  }
}

}  // namespace

void small_spd_solve(bkts_ctx ctx, int k, const double* G, const double* S, double sign, double eps, double* out,
                     int* ndefl) {
  BKTS_REQUIRE(k >= 1 && k <= KM, "k out of range");
  ProfScope prof(ctx, BKTS_K_SMALL, 8.0 * 3 * k * k);
  hipLaunchKernelGGL(spd_solve_kernel, dim3(1), dim3(64), 0, ctx->stream, k, G, S, sign, eps, out, ndefl);
  BKTS_HIP(hipGetLastError());
}

}  // namespace bkts

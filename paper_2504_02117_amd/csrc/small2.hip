// Single-workgroup k x k (and small block-Hessenberg) kernels for block GMRES and block BiCGStab.
// Every coefficient stays on the device in FP64.
#include <algorithm>

#include "devcommon.hpp"
#include "internal.hpp"

namespace bkts {
namespace {

constexpr int KM = BKTS_MAX_K;

// CholQR factor of a Gram matrix G = W^T W (k x k, row-major, device):
//   Rinv = D^-1/2 L^-T, R = L^T D^1/2   with D = diag(G) and L L^T the truncated Cholesky
// factor of D^-1/2 G D^-1/2 (pivots below eps drop their direction: zero column in Rinv, zero row in R).
// Then W Rinv has orthonormal active columns and W ~= (W Rinv) R.
__global__ __launch_bounds__(64) void cholqr_kernel(int k, const double* __restrict__ Gin, double eps,
                                                    double* __restrict__ Rinv, double* __restrict__ R, int* ndefl) {
  __shared__ double L[KM][KM + 1];
  __shared__ double Li[KM][KM + 1];
  __shared__ double sc[KM];
  __shared__ int act[KM];
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
    act[t] = ok;
  }
  __syncthreads();
  for (int e = t; e < k * k; e += 64) {
    const int i = e / k, j = e % k;
    L[i][j] *= sc[i] * sc[j];
  }
  __syncthreads();
  for (int j = 0; j < k; ++j) {
    if (t == 0) {
      const double p = L[j][j];
      if (!act[j] || !(p > eps)) {
        act[j] = 0;
        L[j][j] = 1.0;
      } else {
        L[j][j] = sqrt(p);
      }
    }
    __syncthreads();
    const bool aj = act[j];
    for (int i = j + 1 + t; i < k; i += 64) L[i][j] = aj ? L[i][j] / L[j][j] : 0.0;
    __syncthreads();
    if (aj)
      for (int e = t; e < k * k; e += 64) {
        const int i = e / k, l = e % k;
        if (i > j && l > j && l <= i) L[i][l] -= L[i][j] * L[l][j];
      }
    __syncthreads();
  }
  // Li = L^-1 (lower triangular), column c by thread c, deflated rows/columns zero
  if (t < k) {
    const int c = t;
    for (int i = 0; i < k; ++i) {
      double v = (i == c) ? 1.0 : 0.0;
      for (int l = c; l < i; ++l) v -= L[i][l] * Li[l][c];
      Li[i][c] = (act[i] && act[c] && i >= c) ? v / L[i][i] : 0.0;
    }
  }
  __syncthreads();
  for (int e = t; e < k * k; e += 64) {
    const int i = e / k, j = e % k;
    // Rinv[i][j] = sc[i] * Li[j][i]  (D^-1/2 L^-T);  R[i][j] = L[j][i] / sc[j]  (L^T D^1/2)
    Rinv[i * k + j] = sc[i] * Li[j][i];
    R[i * k + j] = (act[i] && j >= i && sc[j] > 0.0) ? L[j][i] / sc[j] : 0.0;
  }
  if (t == 0 && ndefl) {
    int nd = 0;
    for (int i = 0; i < k; ++i) nd += act[i] ? 0 : 1;
    *ndefl = nd;
  }
}

// C = A * B  (k x k, row-major); alpha scales the product
__global__ __launch_bounds__(256) void small_gemm_kernel(int k, const double* A, const double* B, double alpha,
                                                         double* C) {
  for (int e = threadIdx.x; e < k * k; e += 256) {
    const int i = e / k, j = e % k;
    double s = 0.0;
    for (int l = 0; l < k; ++l) s = fma(A[i * k + l], B[l * k + j], s);
    C[e] = alpha * s;
  }
}

// Solve M X1 = s1 B1 and M X2 = s2 B2 (k x k, row-major) by LU with partial pivoting (thread c owns
// right-hand-side column c of both systems).  Singular pivots (|p| <= eps * max|M|) drop the unknown.
__global__ __launch_bounds__(64) void lu_solve2_kernel(int k, const double* __restrict__ M, const double* B1,
                                                       double s1, double* X1, const double* B2, double s2, double* X2,
                                                       double eps) {
  __shared__ double A[KM][KM + 1];
  __shared__ double Y[2 * KM][KM + 1];
  __shared__ int piv[KM];
  __shared__ int ok[KM];
  __shared__ double amax;
  const int t = threadIdx.x;
  for (int e = t; e < k * k; e += 64) A[e / k][e % k] = M[e];
  __syncthreads();
  if (t == 0) {
    double m = 0.0;
    for (int e = 0; e < k * k; ++e) m = fmax(m, fabs(A[e / k][e % k]));
    amax = m;
  }
  __syncthreads();
  for (int j = 0; j < k; ++j) {
    if (t == 0) {
      int p = j;
      double best = fabs(A[j][j]);
      for (int i = j + 1; i < k; ++i)
        if (fabs(A[i][j]) > best) {
          best = fabs(A[i][j]);
          p = i;
        }
      piv[j] = p;
      ok[j] = best > eps * amax;
      if (p != j)
        for (int l = 0; l < k; ++l) {
          const double tmp = A[j][l];
          A[j][l] = A[p][l];
          A[p][l] = tmp;
        }
    }
    __syncthreads();
    if (ok[j])
      for (int i = j + 1 + t; i < k; i += 64) A[i][j] /= A[j][j];
    __syncthreads();
    if (ok[j])
      for (int e = t; e < k * k; e += 64) {
        const int i = e / k, l = e % k;
        if (i > j && l > j) A[i][l] -= A[i][j] * A[j][l];
      }
    __syncthreads();
  }
  if (t < 2 * k) {
    const int sys = t / k, c = t % k;
    const double* B = sys == 0 ? B1 : B2;
    const double s = sys == 0 ? s1 : s2;
    double* X = sys == 0 ? X1 : X2;
    if (B && X) {
      double y[KM];
      for (int i = 0; i < k; ++i) y[i] = s * B[i * k + c];
      for (int j = 0; j < k; ++j) {  // apply the row swaps in order
        const int p = piv[j];
        const double tmp = y[j];
        y[j] = y[p];
        y[p] = tmp;
      }
      for (int i = 0; i < k; ++i)
        for (int l = 0; l < i; ++l) y[i] -= A[i][l] * y[l];
      for (int i = k - 1; i >= 0; --i) {
        for (int l = i + 1; l < k; ++l) y[i] -= A[i][l] * y[l];
        y[i] = ok[i] ? y[i] / A[i][i] : 0.0;
      }
      for (int i = 0; i < k; ++i) X[i * k + c] = y[i];
    }
    (void)Y;
  }
}

// omega = trace(TS) / trace(TT) for two k x k Grams (scalar; 0 if the denominator vanishes)
__global__ void omega_kernel(int k, const double* TS, const double* TT, double* out) {
  if (threadIdx.x != 0) return;
  double a = 0.0, b = 0.0;
  for (int i = 0; i < k; ++i) {
    a += TS[i * k + i];
    b += TT[i * k + i];
  }
  out[0] = b > 0.0 ? a / b : 0.0;
}

__global__ void diag_ratio_kernel(int k, const double* a, const double* b, double sign, double* out) {
  for (int e = threadIdx.x; e < k * k; e += blockDim.x) {
    const int i = e / k, j = e % k;
    double v = 0.0;
    if (i == j) {
      const double q = sign * a[i] / b[i];
      v = (b[i] != 0.0 && isfinite(q)) ? q : 0.0;
    }
    out[e] = v;
  }
}

// Block upper Hessenberg least squares of block GMRES, min || [S; 0] - H Y ||_F, by Householder QR
// updated one block column per iteration.  H has block lower bandwidth k, so the reflector that
// annihilates the sub-diagonal of column c = jb k + i spans rows c .. (jb + 2)k - 1 (2k - i rows).
// State kept in device memory between calls: the triangular factor Rq (column-major, ldh), the
// reflectors Vr (2k entries per column) with Br = 2 / v^T v (0 = identity), and Gq = Q^T [S; 0]
// (row-major, k columns).  Columns of R whose diagonal is below eps * max|diag| are dropped by the
// back substitution (their unknowns are set to zero), which covers directions deflated by CholQR.
constexpr int kLsqRows = 512;        // rows of the Hessenberg system
constexpr int kLsqLdsDoubles = 8000;  // dynamic LDS of one step: the new block column (jb + 2)k x k plus 2k x k rows of Gq

// Threads per column: a power of two with tpc * k <= 256, at most one wavefront.
__device__ __forceinline__ int lsq_tpc(int k) {
  int t = 64;
  while (t * k > 256 && t > 1) t >>= 1;
  return t;
}

// Sum over the tpc consecutive lanes of a group (tpc divides the wavefront).
__device__ __forceinline__ double group_sum(double v, int tpc) {
  for (int off = tpc >> 1; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

// Block column jb: apply the earlier reflectors, compute k new ones, update Gq and the residual
// norms ||rows (jb+1)k .. (jb+2)k-1 of Gq|| per right-hand side.  Row r of every column is touched
// only by lane r % tpc of that column's group, so the reflector chain needs no barrier.
__global__ __launch_bounds__(256) void gmres_qr_kernel(int k, int jb, const double* __restrict__ H, int ldh,
                                                       const double* __restrict__ S, double* __restrict__ Rq,
                                                       double* __restrict__ Vr, double* __restrict__ Br,
                                                       double* __restrict__ Gq, double* __restrict__ resn) {
  extern __shared__ double lds[];
  __shared__ double vs[2 * KM];
  __shared__ double bs;
  const int nr = (jb + 2) * k, k2 = 2 * k, c0 = jb * k;
  double* B = lds;            // nr x k: the new block column, B[r * k + i]
  double* Gl = lds + nr * k;  // rows c0 .. c0 + 2k - 1 of Gq
  const int t = threadIdx.x;
  const int tpc = lsq_tpc(k);
  const int col = t / tpc, lane = t % tpc;
  const bool act = col < k;
  for (int e = t; e < nr * k; e += blockDim.x) {
    const int r = e / k, i = e % k;
    B[e] = H[(int64_t)(c0 + i) * ldh + r];
  }
  for (int e = t; e < k2 * k; e += blockDim.x) {
    const int r = e / k, i = e % k;
    Gl[e] = r < k ? (jb == 0 ? S[r * k + i] : Gq[(int64_t)(c0 + r) * k + i]) : 0.0;
  }
  __syncthreads();
  if (act) {
    for (int c = 0; c < c0; ++c) {
      const double beta = Br[c];
      if (beta == 0.0) continue;
      const int L = k2 - c % k;
      const double* v = Vr + (int64_t)c * k2;
      const int r0 = c + ((lane - c % tpc) % tpc + tpc) % tpc;
      double d = 0.0;
      for (int r = r0; r < c + L; r += tpc) d += v[r - c] * B[r * k + col];
      d = beta * group_sum(d, tpc);
      for (int r = r0; r < c + L; r += tpc) B[r * k + col] -= d * v[r - c];
    }
  }
  __syncthreads();
  for (int i = 0; i < k; ++i) {
    const int c = c0 + i;
    const int r0 = c + ((lane - c % tpc) % tpc + tpc) % tpc;
    if (col == i) {
      double ss = 0.0;
      for (int r = r0; r < nr; r += tpc) ss += B[r * k + i] * B[r * k + i];
      ss = group_sum(ss, tpc);
      const double x0 = B[c * k + i];  // same value in every lane of the group
      const double nrm = sqrt(ss);
      const double alpha = x0 >= 0.0 ? -nrm : nrm;
      const double v0 = x0 - alpha;
      const double vn2 = ss - x0 * x0 + v0 * v0;
      const double beta = (nrm > 0.0 && vn2 > 0.0) ? 2.0 / vn2 : 0.0;
      for (int r = r0; r < nr; r += tpc) vs[r - c] = r == c ? v0 : B[r * k + i];
      if (lane == c % tpc && beta != 0.0) B[c * k + i] = alpha;
      if (lane == 0) bs = beta;
    }
    __syncthreads();
    const double beta = bs;
    if (act && beta != 0.0) {
      if (col > i) {
        double d = 0.0;
        for (int r = r0; r < nr; r += tpc) d += vs[r - c] * B[r * k + col];
        d = beta * group_sum(d, tpc);
        for (int r = r0; r < nr; r += tpc) B[r * k + col] -= d * vs[r - c];
      }
      // the same reflector on right-hand side `col`: local rows i .. 2k - 1 of Gl
      const int g0 = i + ((lane - i % tpc) % tpc + tpc) % tpc;
      double d = 0.0;
      for (int r = g0; r < k2; r += tpc) d += vs[r - i] * Gl[r * k + col];
      d = beta * group_sum(d, tpc);
      for (int r = g0; r < k2; r += tpc) Gl[r * k + col] -= d * vs[r - i];
    }
    if (t < k2) Vr[(int64_t)c * k2 + t] = t < k2 - i ? vs[t] : 0.0;
    if (t == 0) Br[c] = beta;
    __syncthreads();
  }
  for (int e = t; e < nr * k; e += blockDim.x) {
    const int r = e / k, i = e % k;
    Rq[(int64_t)(c0 + i) * ldh + r] = r <= c0 + i ? B[e] : 0.0;
  }
  for (int e = t; e < k2 * k; e += blockDim.x) {
    const int r = e / k, i = e % k;
    Gq[(int64_t)(c0 + r) * k + i] = Gl[e];
  }
  if (t < k) {
    double ss = 0.0;
    for (int r = k; r < k2; ++r) ss += Gl[r * k + t] * Gl[r * k + t];
    resn[t] = sqrt(ss);
  }
}

// Y (nc x k, row-major) from R Y = Gq (first nc rows) by back substitution; lane r % tpc of each
// right-hand side's group owns row r of Y and reads only the rows it wrote.
__global__ __launch_bounds__(256) void gmres_backsolve_kernel(int k, int nc, const double* __restrict__ Rq, int ldh,
                                                              const double* __restrict__ Gq, double eps,
                                                              double* __restrict__ Y) {
  __shared__ double red[256];
  const int t = threadIdx.x;
  double m = 0.0;
  for (int i = t; i < nc; i += blockDim.x) m = fmax(m, fabs(Rq[(int64_t)i * ldh + i]));
  red[t] = m;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (t < off) red[t] = fmax(red[t], red[t + off]);
    __syncthreads();
  }
  const double tol = eps * red[0];
  const int tpc = lsq_tpc(k);
  const int col = t / tpc, lane = t % tpc;
  if (col >= k) return;
  for (int i = nc - 1; i >= 0; --i) {
    const int l0 = i + 1 + ((lane - (i + 1) % tpc) % tpc + tpc) % tpc;
    double s = 0.0;
    for (int l = l0; l < nc; l += tpc) s += Rq[(int64_t)l * ldh + i] * Y[(int64_t)l * k + col];
    s = group_sum(s, tpc);
    if (lane == i % tpc) {
      const double rii = Rq[(int64_t)i * ldh + i];
      Y[(int64_t)i * k + col] = fabs(rii) > tol ? (Gq[(int64_t)i * k + col] - s) / rii : 0.0;
    }
  }
}

}  // namespace

void small_cholqr(bkts_ctx ctx, int k, const double* G, double eps, double* Rinv, double* R, int* ndefl) {
  BKTS_REQUIRE(k >= 1 && k <= KM, "k out of range");
  ProfScope prof(ctx, BKTS_K_SMALL, 8.0 * 3 * k * k);
  launch(ctx, cholqr_kernel, dim3(1), dim3(64), 0, k, G, eps, Rinv, R, ndefl);
  BKTS_HIP(hipGetLastError());
}

void small_gemm(bkts_ctx ctx, int k, const double* A, const double* B, double alpha, double* C) {
  ProfScope prof(ctx, BKTS_K_SMALL, 8.0 * 3 * k * k);
  launch(ctx, small_gemm_kernel, dim3(1), dim3(256), 0, k, A, B, alpha, C);
  BKTS_HIP(hipGetLastError());
}

void small_lu_solve2(bkts_ctx ctx, int k, const double* M, const double* B1, double s1, double* X1, const double* B2,
                     double s2, double* X2, double eps) {
  BKTS_REQUIRE(k >= 1 && k <= KM, "k out of range");
  ProfScope prof(ctx, BKTS_K_SMALL, 8.0 * 5 * k * k);
  launch(ctx, lu_solve2_kernel, dim3(1), dim3(64), 0, k, M, B1, s1, X1, B2, s2, X2, eps);
  BKTS_HIP(hipGetLastError());
}

void small_omega(bkts_ctx ctx, int k, const double* TS, const double* TT, double* out) {
  ProfScope prof(ctx, BKTS_K_SMALL, 16.0 * k * k);
  launch(ctx, omega_kernel, dim3(1), dim3(64), 0, k, TS, TT, out);
  BKTS_HIP(hipGetLastError());
}

void small_diag_ratio(bkts_ctx ctx, int k, const double* A, const double* B, double sign, double* out) {
  ProfScope prof(ctx, BKTS_K_SMALL, 24.0 * k);
  launch(ctx, diag_ratio_kernel, dim3(1), dim3(256), 0, k, A, B, sign, out);
  BKTS_HIP(hipGetLastError());
}

int gmres_max_rows(int k) {
  k = std::max(k, 1);
  return std::min(kLsqRows, (kLsqLdsDoubles - 2 * k * k) / k);
}

void gmres_qr_step(bkts_ctx ctx, int k, int jb, const double* H, int ldh, const double* S, double* Rq, double* Vr,
                   double* Br, double* Gq, double* resn) {
  const int nr = (jb + 2) * k;
  BKTS_REQUIRE(k >= 1 && k <= KM && nr <= gmres_max_rows(k) && nr <= ldh, "block Hessenberg system too large");
  const size_t lds = sizeof(double) * ((size_t)nr * k + 2 * (size_t)k * k);
  ProfScope prof(ctx, BKTS_K_SMALL, 8.0 * ((double)nr * k * 3 + 2.0 * jb * k * 2 * k));
  launch(ctx, gmres_qr_kernel, dim3(1), dim3(256), lds, k, jb, H, ldh, S, Rq, Vr, Br, Gq, resn);
  BKTS_HIP(hipGetLastError());
}

void gmres_backsolve(bkts_ctx ctx, int k, int nc, const double* Rq, int ldh, const double* Gq, double eps, double* Y) {
  BKTS_REQUIRE(nc >= 1 && nc <= ldh, "bad block Hessenberg size");
  ProfScope prof(ctx, BKTS_K_SMALL, 8.0 * ((double)nc * nc / 2 + 2.0 * nc * k));
  launch(ctx, gmres_backsolve_kernel, dim3(1), dim3(256), 0, k, nc, Rq, ldh, Gq, eps, Y);
  BKTS_HIP(hipGetLastError());
}

}  // namespace bkts

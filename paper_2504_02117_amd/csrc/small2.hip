// Single-workgroup k x k (and small block-Hessenberg) kernels for block GMRES and block BiCGStab.
// Every coefficient stays on the device in FP64.
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

constexpr int kLsqMax = 64;  // rows of the block Hessenberg system handled in LDS

// Least squares min || [S; 0] - H Y ||_F for the block upper Hessenberg H with nr = (j+2)k rows and
// nc = (j+1)k columns (column-major in device memory with leading dimension ldh), by Householder
// QR in LDS.  Writes Y (nc x k, row-major) and the per-column residual norms (k).  Columns of R
// whose diagonal is below eps * max|diag| are dropped (their unknowns set to zero).
__global__ __launch_bounds__(256) void gmres_lsq_kernel(int k, int nr, int nc, const double* __restrict__ H, int ldh,
                                                        const double* __restrict__ S, double eps, double* Y,
                                                        double* resn) {
  __shared__ double A[kLsqMax][kLsqMax + 1];  // A[row][col]
  __shared__ double Bm[kLsqMax][KM + 1];
  __shared__ double v[kLsqMax];
  __shared__ double red[256];
  __shared__ double beta_s, rmax;
  const int t = threadIdx.x;
  for (int e = t; e < nr * nc; e += 256) {
    const int r = e % nr, c = e / nr;
    A[r][c] = H[(int64_t)c * ldh + r];
  }
  for (int e = t; e < nr * k; e += 256) {
    const int r = e / k, c = e % k;
    Bm[r][c] = r < k ? S[r * k + c] : 0.0;
  }
  __syncthreads();
  for (int j = 0; j < nc; ++j) {
    // Householder vector of column j, rows j..nr-1
    double s = 0.0;
    for (int r = j + t; r < nr; r += 256) s += A[r][j] * A[r][j];
    red[t] = s;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
      if (t < off) red[t] += red[t + off];
      __syncthreads();
    }
    if (t == 0) {
      const double nrm = sqrt(red[0]);
      const double x0 = A[j][j];
      const double alpha = x0 >= 0.0 ? -nrm : nrm;
      const double v0 = x0 - alpha;
      const double vn2 = red[0] - x0 * x0 + v0 * v0;
      beta_s = vn2 > 0.0 ? 2.0 / vn2 : 0.0;
      v[j] = v0;
      A[j][j] = alpha;
    }
    __syncthreads();
    for (int r = j + 1 + t; r < nr; r += 256) v[r] = A[r][j];
    __syncthreads();
    // apply to remaining columns of A and to Bm
    const int ncols = (nc - j - 1) + k;
    for (int cc = t; cc < ncols; cc += 256) {
      const bool isA = cc < nc - j - 1;
      const int col = isA ? j + 1 + cc : cc - (nc - j - 1);
      double d = 0.0;
      for (int r = j; r < nr; ++r) d += v[r] * (isA ? A[r][col] : Bm[r][col]);
      d *= beta_s;
      for (int r = j; r < nr; ++r) {
        if (isA)
          A[r][col] -= d * v[r];
        else
          Bm[r][col] -= d * v[r];
      }
    }
    __syncthreads();
    for (int r = j + 1 + t; r < nr; r += 256) A[r][j] = 0.0;
    __syncthreads();
  }
  if (t == 0) {
    double m = 0.0;
    for (int j = 0; j < nc; ++j) m = fmax(m, fabs(A[j][j]));
    rmax = m;
  }
  __syncthreads();
  if (t < k) {  // back substitution for RHS column t
    const int c = t;
    for (int i = nc - 1; i >= 0; --i) {
      double s = Bm[i][c];
      for (int l = i + 1; l < nc; ++l) s -= A[i][l] * Y[l * k + c];
      Y[i * k + c] = fabs(A[i][i]) > eps * rmax ? s / A[i][i] : 0.0;
    }
    double rr = 0.0;
    for (int r = nc; r < nr; ++r) rr += Bm[r][c] * Bm[r][c];
    resn[c] = sqrt(rr);
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

int gmres_max_rows() { return kLsqMax; }

void gmres_lsq(bkts_ctx ctx, int k, int nr, int nc, const double* H, int ldh, const double* S, double eps, double* Y,
               double* resn) {
  BKTS_REQUIRE(nr <= kLsqMax && nc < nr, "block Hessenberg system too large");
  ProfScope prof(ctx, BKTS_K_SMALL, 8.0 * nr * nc);
  launch(ctx, gmres_lsq_kernel, dim3(1), dim3(256), 0, k, nr, nc, H, ldh, S, eps, Y, resn);
  BKTS_HIP(hipGetLastError());
}

}  // namespace bkts

// Streaming helpers on FP64 vectors and block columns used by the time-stepping loop: window
// initialisation, the pipelining shift, column extraction, linear combinations and AXPY.
#include "devcommon.hpp"
#include "internal.hpp"
#include "vecops.hpp"

namespace bkts {
namespace {

__global__ void broadcast_cols_kernel(int64_t N, int k, const double* y, double* Y, int ld) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N * k) return;
  const int64_t r = i / k;
  Y[r * ld + (i % k)] = y[r];
}

__global__ void copy_col_kernel(int64_t N, double* Y, int ld, int src, int dst) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r < N) Y[r * ld + dst] = Y[r * ld + src];
}

__global__ void extract_col_kernel(int64_t N, const double* Y, int ld, int c, double* out) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r < N) out[r] = Y[r * ld + c];
}

// out = column c of Y, then column c = column src (one pass over the rows).
__global__ void take_and_replace_col_kernel(int64_t N, double* Y, int ld, int c, int src, double* out) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= N) return;
  const double v = Y[r * ld + c], w = Y[r * ld + src];
  out[r] = v;
  Y[r * ld + c] = w;
}

__global__ void lincomb_kernel(int64_t N, LinComb lc, double* out, int ldo) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= N) return;
  double s = 0.0;
  for (int i = 0; i < lc.m; ++i) s = fma(lc.a[i], lc.v[i][r * lc.s[i]], s);
  out[r * ldo] = s;
}

__global__ void axpby_kernel(int64_t n, double a, const double* x, double b, double* y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = fma(a, x[i], b * y[i]);
}

__global__ void jacobi_inverse_kernel(int64_t N, const double* diag, double a, double b, double* dinv) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r < N) dinv[r] = 1.0 / (a + b * diag[r]);
}

template <typename T>
__global__ void scale_rows_kernel(int64_t N, int k, const double* dinv, const T* X, T* Y) {
  // 4 elements 256 apart per thread (contiguous per wavefront); one 64-bit division for the first
  // element's row, the others advance by (256 / k, 256 % k)
  const int64_t n = N * k;
  const int64_t i0 = (int64_t)blockIdx.x * 1024 + threadIdx.x;
  int64_t r = i0 / k;
  int c = (int)(i0 - r * k);
  const int dq = 256 / k, dm = 256 % k;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int64_t i = i0 + (int64_t)e * 256;
    if (i < n) Y[i] = (T)((dinv ? dinv[r] : 1.0) * (double)X[i]);
    r += dq;
    c += dm;
    if (c >= k) {
      c -= k;
      ++r;
    }
  }
}

// Y += sign * s[0] * X with the scalar read from device memory
template <typename T>
__global__ void axpy_ds_kernel(int64_t n, const double* s, double sign, const T* X, T* Y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) Y[i] = (T)fma(sign * s[0], (double)X[i], (double)Y[i]);
}

// H[(r0 + i) + (c0 + j) * ldh] (+)= M[i*k + j]  (store a k x k block into a column-major array)
__global__ void hblock_kernel(int k, const double* M, double* H, int ldh, int r0, int c0, int accumulate) {
  for (int e = threadIdx.x; e < k * k; e += blockDim.x) {
    const int i = e / k, j = e % k;
    double* h = H + (int64_t)(c0 + j) * ldh + (r0 + i);
    *h = accumulate ? *h + M[e] : M[e];
  }
}

inline dim3 grid1(int64_t n) { return dim3((unsigned)((n + 255) / 256)); }

}  // namespace

void broadcast_cols(bkts_ctx ctx, int64_t N, int k, const double* y, double* Y, int ld) {
  if (N * k == 0) return;
  ProfScope prof(ctx, BKTS_K_OTHER, 16.0 * N * k);
  launch(ctx, broadcast_cols_kernel, grid1(N * k), dim3(256), 0, N, k, y, Y, ld);
  BKTS_HIP(hipGetLastError());
}

void copy_col(bkts_ctx ctx, int64_t N, double* Y, int ld, int src, int dst) {
  if (N == 0 || src == dst) return;
  ProfScope prof(ctx, BKTS_K_OTHER, 16.0 * N);
  launch(ctx, copy_col_kernel, grid1(N), dim3(256), 0, N, Y, ld, src, dst);
  BKTS_HIP(hipGetLastError());
}

void take_and_replace_col(bkts_ctx ctx, int64_t N, double* Y, int ld, int c, int src, double* out) {
  if (N == 0) return;
  ProfScope prof(ctx, BKTS_K_OTHER, 32.0 * N);
  launch(ctx, take_and_replace_col_kernel, grid1(N), dim3(256), 0, N, Y, ld, c, src, out);
  BKTS_HIP(hipGetLastError());
}

void extract_col(bkts_ctx ctx, int64_t N, const double* Y, int ld, int c, double* out) {
  if (N == 0) return;
  ProfScope prof(ctx, BKTS_K_OTHER, 16.0 * N);
  launch(ctx, extract_col_kernel, grid1(N), dim3(256), 0, N, Y, ld, c, out);
  BKTS_HIP(hipGetLastError());
}

void lincomb(bkts_ctx ctx, int64_t N, const LinComb& lc, double* out, int ldo) {
  BKTS_REQUIRE(lc.m >= 0 && lc.m <= LinComb::kMax, "too many terms");
  if (N == 0) return;
  ProfScope prof(ctx, BKTS_K_OTHER, 8.0 * N * (lc.m + 1));
  launch(ctx, lincomb_kernel, grid1(N), dim3(256), 0, N, lc, out, ldo);
  BKTS_HIP(hipGetLastError());
}

void jacobi_inverse(bkts_ctx ctx, const bkts_op_s& op, double a, double b, double* dinv) {
  if (op.N == 0) return;
  ProfScope prof(ctx, BKTS_K_OTHER, 16.0 * op.N);
  launch(ctx, jacobi_inverse_kernel, grid1(op.N), dim3(256), 0, op.N, op.diag.as<double>(), a, b,
                     dinv);
  BKTS_HIP(hipGetLastError());
}

void scale_rows(bkts_ctx ctx, int dtype, int64_t N, int k, const double* dinv, const void* X, void* Y) {
  if (N * k == 0) return;
  ProfScope prof(ctx, BKTS_K_OTHER, 2.0 * N * k * esize(dtype) + 8.0 * N);
  if (dtype == BKTS_F64)
    launch(ctx, scale_rows_kernel<double>, grid1((N * k + 3) / 4), dim3(256), 0, N, k, dinv,
                       static_cast<const double*>(X), static_cast<double*>(Y));
  else
    launch(ctx, scale_rows_kernel<float>, grid1((N * k + 3) / 4), dim3(256), 0, N, k, dinv,
                       static_cast<const float*>(X), static_cast<float*>(Y));
  BKTS_HIP(hipGetLastError());
}

void axpy_ds(bkts_ctx ctx, int dtype, int64_t n, const double* s, double sign, const void* X, void* Y) {
  if (n == 0) return;
  ProfScope prof(ctx, BKTS_K_OTHER, 3.0 * n * esize(dtype));
  if (dtype == BKTS_F64)
    launch(ctx, axpy_ds_kernel<double>, grid1(n), dim3(256), 0, n, s, sign,
                       static_cast<const double*>(X), static_cast<double*>(Y));
  else
    launch(ctx, axpy_ds_kernel<float>, grid1(n), dim3(256), 0, n, s, sign,
                       static_cast<const float*>(X), static_cast<float*>(Y));
  BKTS_HIP(hipGetLastError());
}

void hblock(bkts_ctx ctx, int k, const double* M, double* H, int ldh, int r0, int c0, bool accumulate) {
  launch(ctx, hblock_kernel, dim3(1), dim3(256), 0, k, M, H, ldh, r0, c0, (int)accumulate);
  BKTS_HIP(hipGetLastError());
}

void axpby(bkts_ctx ctx, int64_t n, double a, const double* x, double b, double* y) {
  if (n == 0) return;
  ProfScope prof(ctx, BKTS_K_OTHER, 24.0 * n);
  launch(ctx, axpby_kernel, grid1(n), dim3(256), 0, n, a, x, b, y);
  BKTS_HIP(hipGetLastError());
}

}  // namespace bkts

// Fused element-wise steps of the vectorized BiCGStab (krylov2.cpp).  Every coefficient is per
// column (the diagonal of a k x k device matrix), so each step is one streaming pass over N x k
// row-major blocks, with the Jacobi scaling D^-1 applied on the way out:
//   s_step:  S = R - V alpha,            Sh = D^-1 S
//   r_step:  R = S - T omega
//   x_step:  X += Ph alpha + Sh omega
//   p_step:  P = R + (P - V omega) beta,  Ph = D^-1 P
// Arithmetic in FP64, stored in the block type.  Each thread handles 4 elements 256 apart.
#include "devcommon.hpp"
#include "internal.hpp"
#include "vecops.hpp"

namespace bkts {
namespace {

constexpr int kEPT = 4;

// Element e of this thread is i0 + e * 256 (i0 = block base + thread index), so every load of a
// wavefront is contiguous.  Row and column of i0 come from one 64-bit division; a stride of 256
// elements advances them by (256 / k, 256 % k).
struct RowCol {
  int64_t r;
  int c, dq, dm;
  __device__ __forceinline__ RowCol(int64_t i, int k) : r(i / k), c((int)(i - (i / k) * k)), dq(256 / k), dm(256 % k) {}
  __device__ __forceinline__ void step(int k) {
    r += dq;
    c += dm;
    if (c >= k) {
      c -= k;
      ++r;
    }
  }
};

// diag of up to three k x k row-major device matrices into shared memory
__device__ __forceinline__ void load_diags(int k, const double* a, const double* b, const double* c, double* sa,
                                           double* sb, double* sc) {
  if (threadIdx.x < k) {
    const int j = threadIdx.x;
    if (a) sa[j] = a[j * k + j];
    if (b) sb[j] = b[j * k + j];
    if (c) sc[j] = c[j * k + j];
  }
  __syncthreads();
}

template <typename T>
__global__ __launch_bounds__(256) void bicg_s_kernel(int64_t n, int k, const T* __restrict__ R,
                                                     const T* __restrict__ V, const double* al,
                                                     const double* __restrict__ dinv, T* __restrict__ S,
                                                     T* __restrict__ Sh) {
  __shared__ double sa[BKTS_MAX_K];
  load_diags(k, al, nullptr, nullptr, sa, nullptr, nullptr);
  const int64_t i0 = (int64_t)blockIdx.x * (256 * kEPT) + threadIdx.x;
  RowCol rc(i0, k);
#pragma unroll
  for (int e = 0; e < kEPT; ++e, rc.step(k)) {
    const int64_t i = i0 + (int64_t)e * 256;
    if (i < n) {
      const double s = (double)R[i] - sa[rc.c] * (double)V[i];
      S[i] = (T)s;
      Sh[i] = (T)(dinv ? dinv[rc.r] * s : s);
    }
  }
}

template <typename T>
__global__ __launch_bounds__(256) void bicg_r_kernel(int64_t n, int k, const T* __restrict__ S,
                                                     const T* __restrict__ Tv, const double* om, T* __restrict__ R) {
  __shared__ double so[BKTS_MAX_K];
  load_diags(k, om, nullptr, nullptr, so, nullptr, nullptr);
  const int64_t i0 = (int64_t)blockIdx.x * (256 * kEPT) + threadIdx.x;
  RowCol rc(i0, k);
#pragma unroll
  for (int e = 0; e < kEPT; ++e, rc.step(k)) {
    const int64_t i = i0 + (int64_t)e * 256;
    if (i < n) R[i] = (T)((double)S[i] - so[rc.c] * (double)Tv[i]);
  }
}

// With nrm (the squared column norms of the residual this step produced), a column whose norm is
// not finite keeps its iterate.
template <typename T>
__global__ __launch_bounds__(256) void bicg_x_kernel(int64_t n, int k, const T* __restrict__ Ph,
                                                     const T* __restrict__ Sh, const double* al, const double* om,
                                                     const double* nrm, T* __restrict__ X) {
  __shared__ double sa[BKTS_MAX_K], so[BKTS_MAX_K];
  __shared__ int live[BKTS_MAX_K];
  if (threadIdx.x < k) live[threadIdx.x] = nrm ? (int)isfinite(nrm[threadIdx.x]) : 1;
  load_diags(k, al, om, nullptr, sa, so, nullptr);
  const int64_t i0 = (int64_t)blockIdx.x * (256 * kEPT) + threadIdx.x;
  RowCol rc(i0, k);
#pragma unroll
  for (int e = 0; e < kEPT; ++e, rc.step(k)) {
    const int64_t i = i0 + (int64_t)e * 256;
    if (i < n && live[rc.c]) X[i] = (T)((double)X[i] + sa[rc.c] * (double)Ph[i] + so[rc.c] * (double)Sh[i]);
  }
}

// n values from device memory to host memory mapped into the device (coherent pinned memory)
__global__ void publish_kernel(const double* src, int n, double* dst) {
  const int i = threadIdx.x;
  if (i < n) dst[i] = src[i];
}

template <typename T>
__global__ __launch_bounds__(256) void bicg_p_kernel(int64_t n, int k, const T* __restrict__ R,
                                                     const T* __restrict__ V, const double* om, const double* be,
                                                     const double* __restrict__ dinv, T* __restrict__ P,
                                                     T* __restrict__ Ph) {
  __shared__ double so[BKTS_MAX_K], sb[BKTS_MAX_K];
  load_diags(k, om, be, nullptr, so, sb, nullptr);
  const int64_t i0 = (int64_t)blockIdx.x * (256 * kEPT) + threadIdx.x;
  RowCol rc(i0, k);
#pragma unroll
  for (int e = 0; e < kEPT; ++e, rc.step(k)) {
    const int64_t i = i0 + (int64_t)e * 256;
    if (i < n) {
      const double p = (double)R[i] + sb[rc.c] * ((double)P[i] - so[rc.c] * (double)V[i]);
      P[i] = (T)p;
      Ph[i] = (T)(dinv ? dinv[rc.r] * p : p);
    }
  }
}

dim3 grid_ept(int64_t n) { return dim3((unsigned)((n + 256 * kEPT - 1) / (256 * kEPT))); }

struct ColCoef {
  double a[BKTS_MAX_K], b[BKTS_MAX_K];
};

template <typename T>
__global__ __launch_bounds__(256) void col_affine_kernel(int64_t n, int k, const T* __restrict__ B,
                                                         const T* __restrict__ X, T* __restrict__ Y, ColCoef cc) {
  const int64_t i0 = (int64_t)blockIdx.x * (256 * kEPT) + threadIdx.x;
  RowCol rc(i0, k);
#pragma unroll
  for (int e = 0; e < kEPT; ++e, rc.step(k)) {
    const int64_t i = i0 + (int64_t)e * 256;
    if (i < n) {
      const double y = cc.b[rc.c] * (double)Y[i] + cc.a[rc.c] * (double)X[i];
      Y[i] = (T)(B ? (double)B[i] - y : y);
    }
  }
}

}  // namespace

void bicg_s_step(bkts_ctx ctx, int dtype, int64_t N, int k, const void* R, const void* V, const double* al,
                 const double* dinv, void* S, void* Sh) {
  const int64_t n = N * k;
  if (n == 0) return;
  ProfScope prof(ctx, BKTS_K_OTHER, 4.0 * n * esize(dtype) + (dinv ? 8.0 * N : 0.0));
  if (dtype == BKTS_F64)
    launch(ctx, bicg_s_kernel<double>, grid_ept(n), dim3(256), 0, n, k, static_cast<const double*>(R),
           static_cast<const double*>(V), al, dinv, static_cast<double*>(S), static_cast<double*>(Sh));
  else
    launch(ctx, bicg_s_kernel<float>, grid_ept(n), dim3(256), 0, n, k, static_cast<const float*>(R),
           static_cast<const float*>(V), al, dinv, static_cast<float*>(S), static_cast<float*>(Sh));
  BKTS_HIP(hipGetLastError());
}

void bicg_r_step(bkts_ctx ctx, int dtype, int64_t N, int k, const void* S, const void* Tv, const double* om, void* R) {
  const int64_t n = N * k;
  if (n == 0) return;
  ProfScope prof(ctx, BKTS_K_OTHER, 3.0 * n * esize(dtype));
  if (dtype == BKTS_F64)
    launch(ctx, bicg_r_kernel<double>, grid_ept(n), dim3(256), 0, n, k, static_cast<const double*>(S),
           static_cast<const double*>(Tv), om, static_cast<double*>(R));
  else
    launch(ctx, bicg_r_kernel<float>, grid_ept(n), dim3(256), 0, n, k, static_cast<const float*>(S),
           static_cast<const float*>(Tv), om, static_cast<float*>(R));
  BKTS_HIP(hipGetLastError());
}

void bicg_x_step(bkts_ctx ctx, int dtype, int64_t N, int k, const void* Ph, const void* Sh, const double* al,
                 const double* om, const double* nrm, void* X) {
  const int64_t n = N * k;
  if (n == 0) return;
  ProfScope prof(ctx, BKTS_K_OTHER, 4.0 * n * esize(dtype));
  if (dtype == BKTS_F64)
    launch(ctx, bicg_x_kernel<double>, grid_ept(n), dim3(256), 0, n, k, static_cast<const double*>(Ph),
           static_cast<const double*>(Sh), al, om, nrm, static_cast<double*>(X));
  else
    launch(ctx, bicg_x_kernel<float>, grid_ept(n), dim3(256), 0, n, k, static_cast<const float*>(Ph),
           static_cast<const float*>(Sh), al, om, nrm, static_cast<float*>(X));
  BKTS_HIP(hipGetLastError());
}

void publish(bkts_ctx ctx, const double* src, int n, double* dst_mapped) {
  BKTS_REQUIRE(n >= 1 && n <= 256, "publish: 1..256 values");
  launch(ctx, publish_kernel, dim3(1), dim3(256), 0, src, n, dst_mapped);
  BKTS_HIP(hipGetLastError());
}

void bicg_p_step(bkts_ctx ctx, int dtype, int64_t N, int k, const void* R, const void* V, const double* om,
                 const double* be, const double* dinv, void* P, void* Ph) {
  const int64_t n = N * k;
  if (n == 0) return;
  ProfScope prof(ctx, BKTS_K_OTHER, 5.0 * n * esize(dtype) + (dinv ? 8.0 * N : 0.0));
  if (dtype == BKTS_F64)
    launch(ctx, bicg_p_kernel<double>, grid_ept(n), dim3(256), 0, n, k, static_cast<const double*>(R),
           static_cast<const double*>(V), om, be, dinv, static_cast<double*>(P), static_cast<double*>(Ph));
  else
    launch(ctx, bicg_p_kernel<float>, grid_ept(n), dim3(256), 0, n, k, static_cast<const float*>(R),
           static_cast<const float*>(V), om, be, dinv, static_cast<float*>(P), static_cast<float*>(Ph));
  BKTS_HIP(hipGetLastError());
}

void col_affine(bkts_ctx ctx, int dtype, int64_t N, int k, const void* B, const void* X, void* Y, const double* a,
                const double* b) {
  BKTS_REQUIRE(k >= 1 && k <= BKTS_MAX_K, "k out of range");
  ColCoef cc{};
  for (int j = 0; j < k; ++j) {
    cc.a[j] = a[j];
    cc.b[j] = b[j];
  }
  const int64_t n = N * k;
  const dim3 grid((unsigned)((n + 256 * kEPT - 1) / (256 * kEPT)));
  ProfScope prof(ctx, BKTS_K_OTHER, (B ? 4.0 : 3.0) * n * esize(dtype));
  if (dtype == BKTS_F64)
    launch(ctx, (col_affine_kernel<double>), grid, dim3(256), 0, n, k, static_cast<const double*>(B),
           static_cast<const double*>(X), static_cast<double*>(Y), cc);
  else
    launch(ctx, (col_affine_kernel<float>), grid, dim3(256), 0, n, k, static_cast<const float*>(B),
           static_cast<const float*>(X), static_cast<float*>(Y), cc);
  BKTS_HIP(hipGetLastError());
}

}  // namespace bkts

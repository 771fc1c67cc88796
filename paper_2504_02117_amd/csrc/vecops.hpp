// Launchers of the streaming vector helpers (vecops.hip).
#pragma once

#include "internal.hpp"

namespace bkts {

// out[r*ldo] = sum_i a[i] * v[i][r*s[i]]   (up to kMax strided FP64 vectors)
struct LinComb {
  static constexpr int kMax = 10;
  int m = 0;
  double a[kMax];
  const double* v[kMax];
  int s[kMax];
  void add(double coef, const double* vec, int stride) {
    a[m] = coef;
    v[m] = vec;
    s[m] = stride;
    ++m;
  }
};

void broadcast_cols(bkts_ctx ctx, int64_t N, int k, const double* y, double* Y, int ld);
void copy_col(bkts_ctx ctx, int64_t N, double* Y, int ld, int src, int dst);
void extract_col(bkts_ctx ctx, int64_t N, const double* Y, int ld, int c, double* out);
// out = column c of Y; then column c = column src
void take_and_replace_col(bkts_ctx ctx, int64_t N, double* Y, int ld, int c, int src, double* out);
void lincomb(bkts_ctx ctx, int64_t N, const LinComb& lc, double* out, int ldo);
void axpby(bkts_ctx ctx, int64_t n, double a, const double* x, double b, double* y);  // y = a x + b y
// Y = diag(dinv) X for N x k contiguous blocks of type dtype (dinv null: copy)
void scale_rows(bkts_ctx ctx, int dtype, int64_t N, int k, const double* dinv, const void* X, void* Y);
// Per-column affine step of a column-wise operator (contiguous N x k blocks of type dtype):
// Y_j = b[j] Y_j + a[j] X_j, and then Y_j = B_j - Y_j when B is given.  a, b: host arrays of k.
void col_affine(bkts_ctx ctx, int dtype, int64_t N, int k, const void* B, const void* X, void* Y, const double* a,
                const double* b);
// Y += sign * s[0] * X (n elements; s is a device scalar)
void axpy_ds(bkts_ctx ctx, int dtype, int64_t n, const double* s, double sign, const void* X, void* Y);
// Fused per-column steps of the vectorized BiCGStab (bicg.hip); alpha, omega, beta are diagonal
// k x k device matrices, dinv may be null (no preconditioner).
// S = R - V alpha, Sh = D^-1 S
void bicg_s_step(bkts_ctx ctx, int dtype, int64_t N, int k, const void* R, const void* V, const double* al,
                 const double* dinv, void* S, void* Sh);
// R = S - T omega
void bicg_r_step(bkts_ctx ctx, int dtype, int64_t N, int k, const void* S, const void* Tv, const double* om, void* R);
// X += Ph alpha + Sh omega, except in the columns whose squared residual norm nrm[j] is not finite
// (nrm may be null)
void bicg_x_step(bkts_ctx ctx, int dtype, int64_t N, int k, const void* Ph, const void* Sh, const double* al,
                 const double* om, const double* nrm, void* X);
// Copy n <= 256 device values into coherent pinned host memory through its device mapping (one
// kernel store per value, so the host may read them after an event without a system fence).
void publish(bkts_ctx ctx, const double* src, int n, double* dst_mapped);
// P = R + (P - V omega) beta, Ph = D^-1 P
void bicg_p_step(bkts_ctx ctx, int dtype, int64_t N, int k, const void* R, const void* V, const double* om,
                 const double* be, const double* dinv, void* P, void* Ph);
// store (or add) a k x k row-major block into a column-major matrix at (r0, c0)
void hblock(bkts_ctx ctx, int k, const double* M, double* H, int ldh, int r0, int c0, bool accumulate);

}  // namespace bkts

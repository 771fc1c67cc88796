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
void lincomb(bkts_ctx ctx, int64_t N, const LinComb& lc, double* out, int ldo);
void axpby(bkts_ctx ctx, int64_t n, double a, const double* x, double b, double* y);  // y = a x + b y

}  // namespace bkts

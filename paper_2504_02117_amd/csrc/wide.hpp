// FP32 block-CG kernels for wide blocks on the FP32 matrix cores (wide.hip).
#pragma once

#include "internal.hpp"
#include "serve.hpp"

namespace bkts {

// Arguments of one wide-block operation; blocks are N x k row-major with ld = k.
struct WideArgs {
  int64_t N;
  int k;
  float *X, *P, *Q, *R;
  const double* dinv;   // inverse Jacobi diagonal or null
  const double* coef;   // k x k (alpha or beta), FP64 row-major
  const int32_t* rowptr;
  const int32_t* col;
  const float* val;     // CSR FP32 values
  double sa, sb;        // Q = sa P + sb K P
  double *pg, *pt, *pn; // partials [entry][slot]
};

// The wide path serves FP32 blocks with 5 <= k <= 32, padded to 16 or 32 columns.
bool wide_eligible(int dtype, int k);
int wide_kp(int k);

void w_cg_update(bkts_ctx ctx, int64_t N, int k, float* X, const float* P, float* R, const float* Q,
                 const double* alpha, const double* dinv, double* gamma, double* Tm, double* nrm,
                 const CgTail* tail = nullptr);
void w_cg_pupdate(bkts_ctx ctx, int64_t N, int k, float* P, const float* R, const double* beta, const double* dinv);
void w_gram(bkts_ctx ctx, int64_t N, int k, const float* X, const float* Y, double* G,
            const CgTail* tail = nullptr);
void w_spmm_gram(bkts_ctx ctx, const bkts_op_s& op, int k, double alpha, const float* P, double beta, float* Q,
                 double* G);

// Grouped variants over jobs of one padded width 16 nb (nb = 1 or 2).
void gw_spmm_gram(bkts_ctx ctx, int nb, const GJob* jobs, GList l);
void gw_update(bkts_ctx ctx, int nb, const GJob* jobs, GList l);
void gw_pupdate(bkts_ctx ctx, int nb, const GJob* jobs, GList l);

}  // namespace bkts

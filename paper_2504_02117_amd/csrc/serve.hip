// Grouped block-CG kernels: every workgroup of a launch first finds its job (binary search over the
// per-job prefix of workgroups), then runs the same row-tile code as the single-solve kernels on
// that job's blocks.  Each job keeps its own slot count and partial buffers, so its reductions are
// bitwise the same whether it runs alone or packed with others.
#include "devcommon.hpp"
#include "serve.hpp"
#include "spd.hpp"

namespace bkts {
namespace {

using dev::TileGeom;

// Largest i with first[i] <= b (first[0] = 0, strictly increasing).
__device__ __forceinline__ int find_job(const int* first, int n, int b) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (first[mid] <= b) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

template <int KP>
constexpr int g_lds(int ntiles) {
  return (ntiles * TileGeom<KP>::LDS_DOUBLES > 4 * KP * KP) ? ntiles * TileGeom<KP>::LDS_DOUBLES : 4 * KP * KP;
}

__device__ __forceinline__ double dinv_at(const double* d, int64_t r) { return d ? d[r] : 1.0; }

template <int KP>
__device__ __forceinline__ void load_col(const double* M, int k, int c, double (&col)[KP]) {
#pragma unroll
  for (int j = 0; j < KP; ++j) col[j] = (j < k && c < k) ? M[j * k + c] : 0.0;
}

// Q = a P + b K P (FP32 CSR gather, FP32 accumulation), and the partials of G = P^T Q.
template <int KP>
__global__ __launch_bounds__(256) void g_spmm_gram_kernel(const GJob* __restrict__ jobs, const int* ids,
                                                          const int* first, int n) {
  using G = TileGeom<KP>;
  __shared__ __align__(16) double lds[g_lds<KP>(1)];
  const int gi = find_job(first, n, blockIdx.x);
  const GJob& J = jobs[ids[gi]];
  const int64_t slot = blockIdx.x - first[gi];
  const int t = threadIdx.x, c = t % KP, r0 = t / KP;
  const int k = J.k;
  const int64_t N = J.N;
  const int64_t ntiles = (N + G::RT - 1) / G::RT;
  const float a = (float)J.a, b = (float)J.b;
  double acc[KP];
#pragma unroll
  for (int e = 0; e < KP; ++e) acc[e] = 0.0;
  const int64_t tend = (slot + 1) * J.tps < ntiles ? (slot + 1) * J.tps : ntiles;
  for (int64_t tile = slot * J.tps; tile < tend; ++tile) {
    const int64_t row0 = tile * G::RT;
    double q[G::RPT];
#pragma unroll
    for (int i = 0; i < G::RPT; ++i) {
      const int row = r0 + i * G::RS;
      const int64_t gr = row0 + row;
      const bool ok = gr < N && c < k;
      float p = 0.f, s = 0.f;
      if (ok) {
        p = J.P[gr * k + c];
        for (int32_t e = J.rowptr[gr]; e < J.rowptr[gr + 1]; ++e) s = fmaf(J.val[e], J.P[(int64_t)J.col[e] * k + c], s);
      }
      const float qv = fmaf(a, p, b * s);
      if (ok) J.Q[gr * k + c] = qv;
      lds[row * G::LDL + c] = p;
      q[i] = ok ? (double)qv : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < G::RPT; ++i) dev::lds_row_axpy<KP>(lds, r0 + i * G::RS, q[i], acc);
    __syncthreads();
  }
  dev::block_reduce_store<KP, KP>(acc, lds, J.pg, J.nslots, slot);
}

// X += P alpha; R -= Q alpha; Z = Dinv R; partials of gamma = R^T Z, T = Q^T Z, nrm = diag(R^T R).
template <int KP>
__global__ __launch_bounds__(256) void g_update_kernel(const GJob* __restrict__ jobs, const int* ids, const int* first,
                                                       int n) {
  using G = TileGeom<KP>;
  __shared__ __align__(16) double lds[g_lds<KP>(2)];
  double* Pl = lds;
  double* Ql = lds + G::LDS_DOUBLES;
  const int gi = find_job(first, n, blockIdx.x);
  const GJob& J = jobs[ids[gi]];
  const int64_t slot = blockIdx.x - first[gi];
  const int t = threadIdx.x, c = t % KP, r0 = t / KP;
  const int k = J.k;
  const int64_t N = J.N;
  const int64_t ntiles = (N + G::RT - 1) / G::RT;
  double acol[KP];
  load_col<KP>(J.alpha, k, c, acol);
  double gacc[KP], tacc[KP], nacc[1] = {0.0};
#pragma unroll
  for (int e = 0; e < KP; ++e) gacc[e] = tacc[e] = 0.0;
  const int64_t tend = (slot + 1) * J.tps < ntiles ? (slot + 1) * J.tps : ntiles;
  for (int64_t tile = slot * J.tps; tile < tend; ++tile) {
    const int64_t row0 = tile * G::RT;
    double x[G::RPT], r[G::RPT], z[G::RPT];
#pragma unroll
    for (int i = 0; i < G::RPT; ++i) {
      const int row = r0 + i * G::RS;
      const int64_t gr = row0 + row;
      const bool ok = gr < N && c < k;
      const int64_t e = gr * k + c;
      Pl[row * G::LDL + c] = ok ? (double)J.P[e] : 0.0;
      Ql[row * G::LDL + c] = ok ? (double)J.Q[e] : 0.0;
      x[i] = ok ? (double)J.X[e] : 0.0;
      r[i] = ok ? (double)J.R[e] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < G::RPT; ++i) {
      const int row = r0 + i * G::RS;
      const int64_t gr = row0 + row;
      const bool ok = gr < N && c < k;
      x[i] += dev::lds_row_dot<KP>(Pl, row, acol);
      r[i] -= dev::lds_row_dot<KP>(Ql, row, acol);
      if (ok) {
        const float xf = (float)x[i], rf = (float)r[i];
        J.X[gr * k + c] = xf;
        J.R[gr * k + c] = rf;
        r[i] = rf;  // the Gram epilogue sees the stored FP32 residual
        z[i] = rf * dinv_at(J.dinv, gr);
      } else {
        r[i] = 0.0;
        z[i] = 0.0;
      }
      nacc[0] = fma(r[i], r[i], nacc[0]);
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < G::RPT; ++i) Pl[(r0 + i * G::RS) * G::LDL + c] = r[i];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < G::RPT; ++i) {
      const int row = r0 + i * G::RS;
      dev::lds_row_axpy<KP>(Pl, row, z[i], gacc);
      dev::lds_row_axpy<KP>(Ql, row, z[i], tacc);
    }
    __syncthreads();
  }
  dev::block_reduce_store<KP, KP>(gacc, lds, J.pg, J.nslots, slot);
  dev::block_reduce_store<KP, KP>(tacc, lds, J.pt, J.nslots, slot);
  dev::block_reduce_store<KP, 1>(nacc, lds, J.pn, J.nslots, slot);
}

// P = Dinv R + P beta
template <int KP>
__global__ __launch_bounds__(256) void g_pupdate_kernel(const GJob* __restrict__ jobs, const int* ids,
                                                        const int* first, int n) {
  using G = TileGeom<KP>;
  __shared__ __align__(16) double lds[g_lds<KP>(1)];
  const int gi = find_job(first, n, blockIdx.x);
  const GJob& J = jobs[ids[gi]];
  const int64_t slot = blockIdx.x - first[gi];
  const int t = threadIdx.x, c = t % KP, r0 = t / KP;
  const int k = J.k;
  const int64_t N = J.N;
  const int64_t ntiles = (N + G::RT - 1) / G::RT;
  double bcol[KP];
  load_col<KP>(J.beta, k, c, bcol);
  const int64_t tend = (slot + 1) * J.tps < ntiles ? (slot + 1) * J.tps : ntiles;
  for (int64_t tile = slot * J.tps; tile < tend; ++tile) {
    const int64_t row0 = tile * G::RT;
    double z[G::RPT];
#pragma unroll
    for (int i = 0; i < G::RPT; ++i) {
      const int row = r0 + i * G::RS;
      const int64_t gr = row0 + row;
      const bool ok = gr < N && c < k;
      lds[row * G::LDL + c] = ok ? (double)J.P[gr * k + c] : 0.0;
      z[i] = ok ? (double)J.R[gr * k + c] * dinv_at(J.dinv, gr) : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < G::RPT; ++i) {
      const int row = r0 + i * G::RS;
      const int64_t gr = row0 + row;
      if (gr < N && c < k) J.P[gr * k + c] = (float)(z[i] + dev::lds_row_dot<KP>(lds, row, bcol));
    }
    __syncthreads();
  }
}

// Fixed-order fold of partials into k x k results (and norms); one workgroup per output entry.
__global__ __launch_bounds__(256) void g_finalize_kernel(const GJob* __restrict__ jobs, const int* ids,
                                                         const int* first, int n, int mode) {
  __shared__ double s[256];
  const int gi = find_job(first, n, blockIdx.x);
  const GJob& J = jobs[ids[gi]];
  int i = blockIdx.x - first[gi];
  const int k = J.k, kk = k * k;
  const double* part;
  double* out;
  int e;
  if (mode == 0) {
    part = J.pg;
    out = J.G + i;
    e = (i / k) * J.kp + i % k;
  } else if (i < kk) {
    part = J.pg;
    out = J.gamma + i;
    e = (i / k) * J.kp + i % k;
  } else if (i < 2 * kk) {
    i -= kk;
    part = J.pt;
    out = J.T + i;
    e = (i / k) * J.kp + i % k;
  } else {
    i -= 2 * kk;
    part = J.pn;
    out = J.nrm + i;
    e = i;
  }
  const double* p = part + (int64_t)e * J.nslots;
  double acc = 0.0;
  for (int j = threadIdx.x; j < J.nslots; j += 256) acc += p[j];
  s[threadIdx.x] = acc;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) s[threadIdx.x] += s[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = s[0];
}

__global__ __launch_bounds__(256) void g_solve_kernel(const GJob* __restrict__ jobs, const int* ids, int mode,
                                                     double eps) {
  __shared__ dev::SolveLds sm;
  const GJob& J = jobs[ids[blockIdx.x]];
  if (mode == 0)
    dev::spd_solve_dev(J.k, J.G, J.gamma, 1.0, eps, J.alpha, J.ndefl, sm);
  else
    dev::spd_solve_dev(J.k, J.G, J.T, -1.0, eps, J.beta, nullptr, sm);
}

__global__ void scales_kernel(int k, const double* nrm2, double* sc, double* sp) {
  const int j = threadIdx.x;
  if (j >= k) return;
  const double s = nrm2[j] > 0.0 ? sqrt(nrm2[j]) : 1.0;
  sc[j] = -s;
  sp[j] = s;
}

}  // namespace

int gjob_slots(int64_t N, int kp, int64_t* tps) {
  if (kp >= 16) {  // matrix-core kernels: 16-row tiles, about eight per workgroup
    const int64_t t16 = (N + 15) / 16;
    int64_t ns = (t16 + 7) / 8;
    ns = ns < 1 ? 1 : (ns > 1024 ? 1024 : ns);
    *tps = (t16 + ns - 1) / ns;
    return (int)ns;
  }
  const int64_t rt = 2048 / kp;
  const int64_t ntiles = (N + rt - 1) / rt;
  int64_t ns = ntiles < 512 ? ntiles : 512;
  if (ns < 1) ns = 1;
  *tps = (ntiles + ns - 1) / ns;
  return (int)ns;
}

#define BKTS_KP_SWITCH(kp, CALL)                 \
  switch (kp) {                                  \
    case 1: { constexpr int KP = 1; CALL; } break;   \
    case 2: { constexpr int KP = 2; CALL; } break;   \
    case 4: { constexpr int KP = 4; CALL; } break;   \
    case 8: { constexpr int KP = 8; CALL; } break;   \
    case 16: { constexpr int KP = 16; CALL; } break; \
    default: { constexpr int KP = 32; CALL; } break; \
  }

void g_spmm_gram(bkts_ctx ctx, int kp, const GJob* jobs, GList l) {
  if (l.n == 0 || l.total == 0) return;
  BKTS_KP_SWITCH(kp, (launch(ctx, g_spmm_gram_kernel<KP>, dim3(l.total), dim3(256), 0, jobs, l.ids, l.first, l.n)));
  BKTS_HIP(hipGetLastError());
}

void g_update(bkts_ctx ctx, int kp, const GJob* jobs, GList l) {
  if (l.n == 0 || l.total == 0) return;
  BKTS_KP_SWITCH(kp, (launch(ctx, g_update_kernel<KP>, dim3(l.total), dim3(256), 0, jobs, l.ids, l.first, l.n)));
  BKTS_HIP(hipGetLastError());
}

void g_pupdate(bkts_ctx ctx, int kp, const GJob* jobs, GList l) {
  if (l.n == 0 || l.total == 0) return;
  BKTS_KP_SWITCH(kp, (launch(ctx, g_pupdate_kernel<KP>, dim3(l.total), dim3(256), 0, jobs, l.ids, l.first, l.n)));
  BKTS_HIP(hipGetLastError());
}

void g_finalize(bkts_ctx ctx, int mode, const GJob* jobs, GList l) {
  if (l.n == 0 || l.total == 0) return;
  launch(ctx, g_finalize_kernel, dim3(l.total), dim3(256), 0, jobs, l.ids, l.first, l.n, mode);
  BKTS_HIP(hipGetLastError());
}

void g_solve(bkts_ctx ctx, int mode, double eps, const GJob* jobs, GList l) {
  if (l.n == 0) return;
  launch(ctx, g_solve_kernel, dim3(l.n), dim3(dev::kSolveThreads), 0, jobs, l.ids, mode, eps);
  BKTS_HIP(hipGetLastError());
}

void scales_from_norms(bkts_ctx ctx, int k, const double* nrm2, double* sc, double* sp) {
  launch(ctx, scales_kernel, dim3(1), dim3(64), 0, k, nrm2, sc, sp);
  BKTS_HIP(hipGetLastError());
}

}  // namespace bkts

// Grouped block-CG kernels for the serving loop (serve.hip): one launch advances every resident
// solve of a block-width class by one step of the iteration.
#pragma once

#include <vector>

#include "internal.hpp"

namespace bkts {

// Device-side descriptor of one resident FP32 block-CG solve of (a I + b K) X = R.  Blocks are
// N x k, row-major, ld = k.  Partials are laid out [entry][slot] with `nslots` slots, the same for
// every launch of this job, so a job's arithmetic does not depend on which other jobs share a launch.
struct GJob {
  int64_t N;
  int k, kp, nslots;
  int64_t tps;  // row tiles per slot
  double a, b;
  const int32_t* rowptr;
  const int32_t* col;
  const float* val;
  const double* dinv;
  float *X, *P, *Q, *R;
  double *G, *gamma, *T, *alpha, *beta, *nrm;
  int* ndefl;
  double *pg, *pt, *pn;
};

// Number of reduction slots of a job: fixed by (N, KP) alone.
int gjob_slots(int64_t N, int kp, int64_t* tps);

// One grouped launch list: `ids` index the device job table; `first[i]` is the first workgroup
// (or entry) of job ids[i]; `first[n]` is the total.
struct GList {
  const int* ids;
  const int* first;
  int n;
  int total;
};

// Grouped launches (all on ctx->stream).
void g_spmm_gram(bkts_ctx ctx, int kp, const GJob* jobs, GList l);
void g_update(bkts_ctx ctx, int kp, const GJob* jobs, GList l);
void g_pupdate(bkts_ctx ctx, int kp, const GJob* jobs, GList l);
// mode 0: G from pg; mode 1: gamma, T, nrm from pg, pt, pn.  `l.first` counts output entries.
void g_finalize(bkts_ctx ctx, int mode, const GJob* jobs, GList l);
// mode 0: alpha = G^+ gamma (and ndefl); mode 1: beta = -G^+ T.  One workgroup per job.
void g_solve(bkts_ctx ctx, int mode, double eps, const GJob* jobs, GList l);

// Per-job helpers of the outer loop.
// sc[j] = -||R_j|| (1 when zero), sp[j] = -sc[j]: R32 = R64 / sc, Y += X * sp applies Y -= J^-1 R.
void scales_from_norms(bkts_ctx ctx, int k, const double* nrm2, double* sc, double* sp);

}  // namespace bkts

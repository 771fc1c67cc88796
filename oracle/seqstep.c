/*
 * Sequential implicit Euler for y' + K y = b, one Jacobi-preconditioned CG solve per step.
 * Plain C, FP64 (part of the CPU oracle).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the benchmark's CPU-baseline
 * leg, never by the HIP library or its binding.  It shares no code with the HIP path.
 *
 * What it computes is the plain definition the all-at-once block method must reproduce: step by
 * step time integration (Sec. 2.1, eq. general-system-time-steps, is the stages stacked; for
 * implicit Euler, the tableau A = [1] of eq. stiffly-accurate-DIRK), with M = I:
 *
 *     (I/tau + K) y^{n+1} = y^n / tau + b.
 *
 * Each step is solved by the textbook preconditioned conjugate-gradient method with the diagonal of
 * J = I/tau + K as preconditioner, from the initial guess y^n, until the true residual meets
 * ||rhs - J y||_2 <= rtol ||rhs||_2.  K is a CSR matrix (int32 indices) assembled by the Python
 * oracle.  The loops over rows are split over OpenMP threads with a static schedule, so a given
 * thread count always sums in the same order.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* y = s x + K x */
static void jmul(int64_t N, const int32_t* rp, const int32_t* ci, const double* v, double s, const double* x,
                 double* y) {
#pragma omp parallel for schedule(static)
  for (int64_t r = 0; r < N; ++r) {
    double acc = s * x[r];
    for (int32_t e = rp[r]; e < rp[r + 1]; ++e) acc += v[e] * x[ci[e]];
    y[r] = acc;
  }
}

static double dot(int64_t N, const double* a, const double* b) {
  double s = 0.0;
#pragma omp parallel for reduction(+ : s) schedule(static)
  for (int64_t i = 0; i < N; ++i) s += a[i] * b[i];
  return s;
}

/* PCG on J x = rhs with J = s I + K and D^-1 = dinv.  Returns iterations, or -1 without convergence
 * within maxit.  The recursive residual drives the loop; the true residual is checked at the end
 * and the iteration restarted from x if it has drifted above the tolerance. */
static int pcg(int64_t N, const int32_t* rp, const int32_t* ci, const double* v, double s, const double* dinv,
               const double* rhs, double* x, double rtol, int maxit, double* r, double* z, double* p, double* q) {
  const double tol = rtol * sqrt(dot(N, rhs, rhs));
  int its = 0;
  for (int attempt = 0; attempt < 8; ++attempt) {
    jmul(N, rp, ci, v, s, x, q);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; ++i) {
      r[i] = rhs[i] - q[i];
      z[i] = dinv[i] * r[i];
      p[i] = z[i];
    }
    if (sqrt(dot(N, r, r)) <= tol) return its;
    double rz = dot(N, r, z);
    int met = 0;
    while (its < maxit) {
      jmul(N, rp, ci, v, s, p, q);
      const double alpha = rz / dot(N, p, q);
#pragma omp parallel for schedule(static)
      for (int64_t i = 0; i < N; ++i) {
        x[i] += alpha * p[i];
        r[i] -= alpha * q[i];
      }
      ++its;
      if (sqrt(dot(N, r, r)) <= tol) {
        met = 1;
        break;
      }
#pragma omp parallel for schedule(static)
      for (int64_t i = 0; i < N; ++i) z[i] = dinv[i] * r[i];
      const double rz1 = dot(N, r, z);
      const double beta = rz1 / rz;
      rz = rz1;
#pragma omp parallel for schedule(static)
      for (int64_t i = 0; i < N; ++i) p[i] = z[i] + beta * p[i];
    }
    if (!met) return -1;
  }
  return -1;
}

/*
 * Take n_steps implicit Euler steps of size tau from y0 (length N).  ys (n_steps x N, row-major)
 * receives y^1 .. y^{n_steps}; iters (n_steps, may be NULL) the CG iterations of each step.
 * nthreads > 0 fixes the OpenMP thread count, 0 keeps the runtime's default.  *threads_used (may
 * be NULL) returns the count used.  Returns 0, or the 1-based step whose solve did not converge
 * within maxit iterations, or -1 when memory runs out.
 */
int orc_ie_steps(int64_t N, const int32_t* rowptr, const int32_t* col, const double* val, const double* b,
                 double tau, const double* y0, int n_steps, double rtol, int maxit, int nthreads, double* ys,
                 int* iters, int* threads_used) {
  if (nthreads > 0) omp_set_num_threads(nthreads);
  if (threads_used) *threads_used = omp_get_max_threads();
  double* buf = (double*)malloc(sizeof(double) * (size_t)N * 7);
  if (!buf) return -1;
  double *dinv = buf, *rhs = buf + N, *x = buf + 2 * N, *r = buf + 3 * N, *z = buf + 4 * N, *p = buf + 5 * N,
         *q = buf + 6 * N;
  const double s = 1.0 / tau;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < N; ++i) {
    double d = s;
    for (int32_t e = rowptr[i]; e < rowptr[i + 1]; ++e)
      if (col[e] == i) d += val[e];
    dinv[i] = 1.0 / d;
    x[i] = y0[i];
  }
  int status = 0;
  for (int n = 0; n < n_steps; ++n) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; ++i) rhs[i] = s * x[i] + (b ? b[i] : 0.0);
    /* the previous state is the initial guess (x already holds it) */
    const int its = pcg(N, rowptr, col, val, s, dinv, rhs, x, rtol, maxit, r, z, p, q);
    if (iters) iters[n] = its;
    memcpy(ys + (size_t)n * N, x, sizeof(double) * (size_t)N);
    if (its < 0) {
      status = n + 1;
      break;
    }
  }
  free(buf);
  return status;
}

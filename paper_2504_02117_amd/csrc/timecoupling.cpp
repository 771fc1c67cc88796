// Time coupling of a stiffly accurate Runge-Kutta method (Sec. 2, eq. stiffly-accurate-DIRK; Sec.
// 2.1): tableau, elimination of an explicit first stage, and the k x k window matrices A1, A2 of
// eq. time-stepping-matrices-multiple-parallel-time-steps taken from the diagonal position of the
// window's front stage (Sec. 2.2, pipelining).  Fully implicit tableaux (the remark on fully
// implicit Runge-Kutta methods after Algorithm 1) give full diagonal blocks in A2; their windows
// hold whole steps and their splitting uses one averaged coefficient for every stage.
#include <algorithm>
#include <cmath>

#include "internal.hpp"
#include "timecoupling.hpp"

namespace bkts {

// Entry (qi, qj) of the unbounded stage-coupling matrices, with global stage indices counted from
// the first implicit stage of the front step.  A1 = I/tau plus -1/tau from every stage of step
// s >= 1 to the last stage of step s-1 (that stage is y^{n+s}); A2 = block-diagonal implicit
// tableau plus, when an explicit first stage was eliminated, its couplings a_{i,1} at the
// positions of those -1/tau entries.
static void coupling_entry(const bkts_tc_s& tc, int qi, int qj, double& a1, double& a2) {
  const int mi = tc.m_impl;
  const int si = qi / mi, sj = qj / mi;
  const int li = qi % mi, lj = qj % mi;
  a1 = (qi == qj) ? 1.0 / tc.tau : 0.0;
  a2 = (si == sj) ? tc.Ai[li * mi + lj] : 0.0;
  if (si >= 1 && qj == si * mi - 1) {
    a1 += -1.0 / tc.tau;
    if (tc.explicit_first) a2 += tc.ae[li];
  }
}

// |det A|^(1/m) of an m x m row-major matrix (Gaussian elimination with partial pivoting): the
// geometric mean of the moduli of A's eigenvalues.
static double geometric_mean_modulus(std::vector<double> a, int m) {
  double logdet = 0.0;
  for (int c = 0; c < m; ++c) {
    int p = c;
    for (int r = c + 1; r < m; ++r)
      if (std::fabs(a[r * m + c]) > std::fabs(a[p * m + c])) p = r;
    if (a[p * m + c] == 0.0) return 0.0;
    if (p != c)
      for (int j = 0; j < m; ++j) std::swap(a[p * m + j], a[c * m + j]);
    logdet += std::log(std::fabs(a[c * m + c]));
    for (int r = c + 1; r < m; ++r) {
      const double f = a[r * m + c] / a[c * m + c];
      for (int j = c; j < m; ++j) a[r * m + j] -= f * a[c * m + j];
    }
  }
  return std::exp(logdet / m);
}

bkts_tc tc_create(bkts_ctx ctx, const bkts_tc_desc* d) {
  BKTS_REQUIRE(d, "desc must not be NULL");
  BKTS_REQUIRE(d->k >= 1 && d->k <= BKTS_MAX_K, "k must be in 1..%d (got %d)", BKTS_MAX_K, d->k);
  BKTS_REQUIRE(d->tau > 0.0 && std::isfinite(d->tau), "tau must be positive");
  int m = 0;
  std::vector<double> A, c;
  switch (d->method) {
    case BKTS_IE:
      m = 1;
      A = {1.0};
      c = {1.0};
      break;
    case BKTS_THETA:
      BKTS_REQUIRE(d->theta > 0.0 && d->theta <= 1.0, "theta must be in (0, 1]");
      m = 2;
      A = {0.0, 0.0, 1.0 - d->theta, d->theta};
      c = {0.0, 1.0};
      break;
    case BKTS_SDIRK2: {
      const double g = 1.0 - 1.0 / std::sqrt(2.0);
      m = 2;
      A = {g, 0.0, 1.0 - g, g};
      c = {g, 1.0};
      break;
    }
    case BKTS_RADAU2:  // 2-stage Radau IIA: order 3, stiffly accurate, L-stable, fully implicit
      m = 2;
      A = {5.0 / 12.0, -1.0 / 12.0, 0.75, 0.25};
      c = {1.0 / 3.0, 1.0};
      break;
    case BKTS_DIRK_CUSTOM:
      BKTS_REQUIRE(d->stages >= 1 && d->stages <= 8 && d->A && d->c, "custom tableau needs 1..8 stages, A and c");
      m = d->stages;
      A.assign(d->A, d->A + m * m);
      c.assign(d->c, d->c + m);
      for (double v : A) BKTS_REQUIRE(std::isfinite(v), "tableau entries must be finite");
      // a consistent stiffly accurate method: stage times are the row sums of A, and the last
      // stage (the step result, b = last row) ends the step, c_m = 1
      for (int i = 0; i < m; ++i) {
        double rs = 0.0;
        for (int j = 0; j < m; ++j) rs += A[i * m + j];
        BKTS_REQUIRE(std::isfinite(c[i]) && std::fabs(rs - c[i]) <= 1e-12 * std::max(1.0, std::fabs(c[i])),
                     "custom tableau: c_%d = %g is not the row sum %g of A", i + 1, c[i], rs);
      }
      BKTS_REQUIRE(std::fabs(c[m - 1] - 1.0) <= 1e-12, "custom tableau: a stiffly accurate method needs c_m = 1");
      break;
    default:
      throw Error{BKTS_EINVAL, fmt("unknown method %d", d->method)};
  }
  bkts_tc t = new bkts_tc_s();
  t->ctx = ctx;
  t->k = d->k;
  t->tau = d->tau;
  bool expl = true;
  for (int j = 0; j < m; ++j) expl = expl && A[j] == 0.0;
  expl = expl && m > 1;
  t->explicit_first = expl ? 1 : 0;
  const int off = expl ? 1 : 0;
  const int mi = m - off;
  t->m_impl = mi;
  t->Ai.assign(mi * mi, 0.0);
  t->ae.assign(mi, 0.0);
  t->ci.assign(mi, 0.0);
  for (int i = 0; i < mi; ++i) {
    for (int j = 0; j < mi; ++j) t->Ai[i * mi + j] = A[(i + off) * m + (j + off)];
    if (expl) t->ae[i] = A[(i + off) * m];
    t->ci[i] = c[i + off];
  }
  for (int i = 0; i < mi; ++i)
    for (int j = i + 1; j < mi; ++j) t->fully_implicit |= t->Ai[i * mi + j] != 0.0 ? 1 : 0;
  if (t->fully_implicit) {
    t->beta_avg = geometric_mean_modulus(t->Ai, mi);
    if (!(t->beta_avg > 0.0) || d->k % mi != 0) {
      delete t;
      throw Error{BKTS_EINVAL, fmt("a fully implicit tableau needs a nonsingular A and k a multiple of its %d "
                                   "implicit stages (got k=%d)", mi, d->k)};
    }
  } else {
    for (int i = 0; i < mi; ++i) {
      if (!(t->Ai[i * mi + i] > 0.0)) {
        delete t;
        throw Error{BKTS_EINVAL, "implicit stages need a positive diagonal entry"};
      }
    }
  }
  const int k = d->k;
  t->A1.assign(mi, std::vector<double>(k * k));
  t->A2.assign(mi, std::vector<double>(k * k));
  for (int p = 0; p < mi; ++p)
    for (int i = 0; i < k; ++i)
      for (int j = 0; j < k; ++j) coupling_entry(*t, p + i, p + j, t->A1[p][i * k + j], t->A2[p][i * k + j]);
  return t;
}

}  // namespace bkts

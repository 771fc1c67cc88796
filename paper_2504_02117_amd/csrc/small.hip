// k x k dense kernels that run on one workgroup and keep every block-Krylov coefficient on the
// device in FP64: the truncated (deflating) Cholesky solve used by block CG, and helpers.
#include "devcommon.hpp"
#include "internal.hpp"
#include "spd.hpp"

namespace bkts {
namespace {

using dev::SolveLds;
using dev::spd_solve_dev;

__global__ __launch_bounds__(256) void spd_solve_kernel(int k, const double* __restrict__ G,
                                                       const double* __restrict__ S, double sign, double eps,
                                                       double* __restrict__ out, int* ndefl) {
  __shared__ SolveLds sm;
  spd_solve_dev(k, G, S, sign, eps, out, ndefl, sm);
}

}  // namespace

void small_spd_solve(bkts_ctx ctx, int k, const double* G, const double* S, double sign, double eps, double* out,
                     int* ndefl) {
  BKTS_REQUIRE(k >= 1 && k <= dev::KM, "k out of range");
  ProfScope prof(ctx, BKTS_K_SMALL, 8.0 * 3 * k * k);
  launch(ctx, spd_solve_kernel, dim3(1), dim3(dev::kSolveThreads), 0, k, G, S, sign, eps, out, ndefl);
  BKTS_HIP(hipGetLastError());
}


}  // namespace bkts

// Fold + solve in one launch: one workgroup per partial entry sums that entry over the slots in a
// fixed order (as the plain fold), and the workgroup that finishes last (device-scope counter)
// solves the k x k system from the folded values.  MODE 0 follows a Gram kernel (G, then
// alpha = G^+ gamma_in); MODE 1 follows a block-CG update kernel whose partials are laid out
// [gamma (KP^2) | T (KP^2) | nrm (KP)] (gamma, T, nrm, then beta = -G^+ T, and optionally the norms
// and the deflation count of the preceding alpha solve written to pinned host memory).  Entries are
// a*KP + b; rows or columns >= k are padding and are dropped.
#include "devcommon.hpp"
#include "internal.hpp"
#include "spd.hpp"

namespace bkts {
namespace {

template <int KP, int MODE>
__global__ __launch_bounds__(256) void fold_solve_kernel(const double* __restrict__ partials, int64_t nslots, int k,
                                                         CgTail t) {
  constexpr int KK = KP * KP;
  __shared__ double s[256];
  __shared__ dev::SolveLdsT<KP> sm;
  const int e = blockIdx.x;
  const double* p = partials + (int64_t)e * nslots;
  double acc = 0.0;
  for (int64_t j = threadIdx.x; j < nslots; j += 256) acc += p[j];
  s[threadIdx.x] = acc;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) s[threadIdx.x] += s[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const int set = e < KK ? 0 : (e < 2 * KK ? 1 : 2);
    const int r = set < 2 ? (e - set * KK) / KP : 0, c = set < 2 ? (e - set * KK) % KP : e - 2 * KK;
    if (r < k && c < k) {
      double* out = MODE == 0 ? t.G : (set == 0 ? t.gamma : (set == 1 ? t.T : t.nrm));
      out[set < 2 ? r * k + c : c] = s[0];
    }
  }
  if (!dev::last_workgroup(t.counter)) return;
  if (MODE == 0) {
    dev::spd_solve_dev_t<KP>(k, t.G, t.gamma_in, 1.0, t.eps, t.alpha, t.ndefl, sm);
  } else {
    dev::spd_solve_dev_t<KP>(k, t.G, t.T, -1.0, t.eps, t.beta, nullptr, sm);
    if (t.host) {
      if (threadIdx.x < k) t.host[threadIdx.x] = t.nrm[threadIdx.x];
      if (threadIdx.x == 0) *reinterpret_cast<int*>(t.host + k) = t.ndefl ? *t.ndefl : 0;
    }
  }
  if (threadIdx.x == 0) atomicExch(t.counter, 0u);
}

template <int KP>
void fold_solve_t(bkts_ctx ctx, int mode, int k, const double* partials, int64_t nslots, const CgTail& t) {
  const int E = mode == 0 ? KP * KP : 2 * KP * KP + KP;
  ProfScope ps(ctx, BKTS_K_SMALL, 8.0 * E * nslots);
  if (mode == 0)
    launch(ctx, (fold_solve_kernel<KP, 0>), dim3(E), dim3(256), 0, partials, nslots, k, t);
  else
    launch(ctx, (fold_solve_kernel<KP, 1>), dim3(E), dim3(256), 0, partials, nslots, k, t);
  BKTS_HIP(hipGetLastError());
}

}  // namespace

void fold_solve(bkts_ctx ctx, int mode, int kp, int k, const double* partials, int64_t nslots, const CgTail& t) {
  BKTS_REQUIRE(t.counter, "fold_solve needs a counter");
  switch (kp) {
    case 1: fold_solve_t<1>(ctx, mode, k, partials, nslots, t); break;
    case 2: fold_solve_t<2>(ctx, mode, k, partials, nslots, t); break;
    case 4: fold_solve_t<4>(ctx, mode, k, partials, nslots, t); break;
    case 16: fold_solve_t<16>(ctx, mode, k, partials, nslots, t); break;
    case 32: fold_solve_t<32>(ctx, mode, k, partials, nslots, t); break;
    default: throw Error{BKTS_EINVAL, fmt("fold_solve: unsupported padded width %d", kp)};
  }
}

}  // namespace bkts

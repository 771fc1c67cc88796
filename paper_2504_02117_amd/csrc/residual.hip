// Fused all-at-once residual R = Y A1^T + (K Y - b 1^T) A2^T - B0 with per-column norms
// (Sec. 2.2; the k x k couplings act from the right, eq. general-system-time-steps with the
// identity (C (x) A) vec X = vec(A X C^T)).  One pass over Y: the sparse product of the tile rows
// is formed in registers and staged in LDS next to the Y tile, both right multiplications read
// whole rows from LDS, and the squared column norms are reduced deterministically.
#include "devcommon.hpp"
#include "internal.hpp"

namespace bkts {
namespace {

using dev::TileGeom;

constexpr int kMaxB0 = 8;

struct ResArgs {
  int64_t N;
  int k;
  const int32_t* rowptr;
  const int32_t* col;
  const double* val;
  const int64_t* sptr;
  const int32_t* sw;
  int C;
  int uw;                 // uniform SELL width (0: per-slice widths)
  int na;                 // stencil form: number of neighbour offsets (0: none)
  int64_t soff[3];
  const double* coef;     // stencil form: diagonal, then one array per offset
  const double* Y;
  int ldy;
  const double* A1;    // row-major k x k (physical column order)
  const double* A2;
  const double* b;     // source or null
  const double* rs;    // row sums of A2 (device, k) used with b
  const double* B0;
  int ldb0, nb0;
  int b0col[kMaxB0];
  double* R;
  int ldr;
  double* partials;
  int64_t tps;
};

template <int KP>
constexpr int res_lds() {
  return (2 * TileGeom<KP>::LDS_DOUBLES > 4 * KP) ? 2 * TileGeom<KP>::LDS_DOUBLES : 4 * KP;
}

// (K Y)[gr, c] for FMT 0 (CSR), 1 (SELL-C) and 2 (stencil form).  Every load of the row is issued
// before the first FMA: the stencil form's addresses are known up front, and a uniform-width SELL
// row issues its (at most 8) value/index loads, then its Y loads.
template <int FMT>
__device__ __forceinline__ double row_ky(const ResArgs& a, int64_t gr, int c) {
  double ky = 0.0;
  if constexpr (FMT == 2) {
    double up[3], lo[3], yu[3], yl[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      up[q] = lo[q] = yu[q] = yl[q] = 0.0;
      if (q < a.na) {
        const int64_t s = a.soff[q];
        const double* oq = a.coef + (1 + q) * a.N;
        if (gr + s < a.N) {
          up[q] = oq[gr];
          yu[q] = a.Y[(gr + s) * a.ldy + c];
        }
        if (gr - s >= 0) {
          lo[q] = oq[gr - s];
          yl[q] = a.Y[(gr - s) * a.ldy + c];
        }
      }
    }
    ky = a.coef[gr] * a.Y[gr * a.ldy + c];
#pragma unroll
    for (int q = 0; q < 3; ++q) ky = fma(up[q], yu[q], fma(lo[q], yl[q], ky));
  } else if constexpr (FMT == 1) {
    const int64_t sl = gr / a.C;
    if (a.uw > 0 && a.uw <= 8) {
      const int64_t base = sl * a.C * a.uw + (gr - sl * a.C);
      double v[8], y[8];
      int32_t ci[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        v[u] = u < a.uw ? a.val[base + (int64_t)u * a.C] : 0.0;
        ci[u] = u < a.uw ? a.col[base + (int64_t)u * a.C] : (int32_t)gr;
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) y[u] = a.Y[(int64_t)ci[u] * a.ldy + c];
#pragma unroll
      for (int u = 0; u < 8; ++u) ky = fma(v[u], y[u], ky);
    } else {
      const int64_t base = a.sptr[sl] + (gr - sl * a.C);
      const int64_t len = a.sw[sl];
      for (int64_t j = 0; j < len; ++j) {
        const int64_t e = base + j * a.C;
        ky = fma(a.val[e], a.Y[(int64_t)a.col[e] * a.ldy + c], ky);
      }
    }
  } else {
    const int64_t base = a.rowptr[gr];
    const int64_t len = a.rowptr[gr + 1] - base;
    for (int64_t j = 0; j < len; ++j) ky = fma(a.val[base + j], a.Y[(int64_t)a.col[base + j] * a.ldy + c], ky);
  }
  return ky;
}

template <int KP, int FMT>
__global__ __launch_bounds__(256) void residual_kernel(ResArgs a) {
  using G = TileGeom<KP>;
  __shared__ __align__(16) double lds[res_lds<KP>()];
  double* Yl = lds;
  double* KYl = lds + G::LDS_DOUBLES;
  const int t = threadIdx.x, c = t % KP, r0 = t / KP;
  const int64_t slot = dev::xcd_slot(blockIdx.x, gridDim.x);
  const int64_t ntiles = (a.N + G::RT - 1) / G::RT;
  const bool cok = c < a.k;
  double a1[KP], a2[KP];
#pragma unroll
  for (int j = 0; j < KP; ++j) {
    a1[j] = (cok && j < a.k) ? a.A1[c * a.k + j] : 0.0;
    a2[j] = (cok && j < a.k) ? a.A2[c * a.k + j] : 0.0;
  }
  const double rsc = (a.b && cok) ? a.rs[c] : 0.0;
  int b0j = -1;
  for (int j = 0; j < a.nb0; ++j)
    if (a.b0col[j] == c) b0j = j;
  double nacc[1] = {0.0};
  const int64_t tend = (slot + 1) * a.tps < ntiles ? (slot + 1) * a.tps : ntiles;
  for (int64_t tile = slot * a.tps; tile < tend; ++tile) {
    const int64_t row0 = tile * G::RT;
#pragma unroll 2
    for (int i = 0; i < G::RPT; ++i) {
      const int row = r0 + i * G::RS;
      const int64_t gr = row0 + row;
      double yv = 0.0, ky = 0.0;
      if (gr < a.N && cok) {
        yv = a.Y[gr * a.ldy + c];
        ky = row_ky<FMT>(a, gr, c);
      }
      Yl[row * G::LDL + c] = yv;
      KYl[row * G::LDL + c] = ky;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < G::RPT; ++i) {
      const int row = r0 + i * G::RS;
      const int64_t gr = row0 + row;
      if (gr < a.N && cok) {
        double r = dev::lds_row_dot<KP>(Yl, row, a1) + dev::lds_row_dot<KP>(KYl, row, a2);
        if (a.b) r -= a.b[gr] * rsc;
        if (b0j >= 0) r -= a.B0[gr * a.ldb0 + b0j];
        a.R[gr * a.ldr + c] = r;
        nacc[0] = fma(r, r, nacc[0]);
      }
    }
    __syncthreads();
  }
  dev::block_reduce_store<KP, 1>(nacc, lds, a.partials, gridDim.x, slot);
}

// Stencil form, k <= 4: one thread per row holds the whole row of Y, of K Y and of R in registers
// (no LDS staging); A1 and A2 sit in registers; the column norms are folded per workgroup.
template <int KP>
__global__ __launch_bounds__(256) void st_residual_row_kernel(ResArgs a) {
  __shared__ double red[4 * KP];
  double a1[KP][KP], a2[KP][KP], rs[KP];
  int b0[KP];
#pragma unroll
  for (int c = 0; c < KP; ++c) {
#pragma unroll
    for (int j = 0; j < KP; ++j) {
      a1[c][j] = a.A1[c * KP + j];
      a2[c][j] = a.A2[c * KP + j];
    }
    rs[c] = a.b ? a.rs[c] : 0.0;
    b0[c] = -1;
    for (int j = 0; j < a.nb0; ++j)
      if (a.b0col[j] == c) b0[c] = j;
  }
  double nacc[KP];
#pragma unroll
  for (int c = 0; c < KP; ++c) nacc[c] = 0.0;
  const int64_t N = a.N;
  for (int64_t r = (int64_t)blockIdx.x * dev::kThreads + threadIdx.x; r < N; r += (int64_t)gridDim.x * dev::kThreads) {
    double y[KP], up[3], lo[3], yu[3][KP], yl[3][KP];
#pragma unroll
    for (int j = 0; j < KP; ++j) y[j] = a.Y[r * a.ldy + j];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      up[q] = lo[q] = 0.0;
#pragma unroll
      for (int j = 0; j < KP; ++j) yu[q][j] = yl[q][j] = 0.0;
      if (q < a.na) {
        const int64_t s = a.soff[q];
        const double* oq = a.coef + (1 + q) * N;
        if (r + s < N) {
          up[q] = oq[r];
#pragma unroll
          for (int j = 0; j < KP; ++j) yu[q][j] = a.Y[(r + s) * a.ldy + j];
        }
        if (r - s >= 0) {
          lo[q] = oq[r - s];
#pragma unroll
          for (int j = 0; j < KP; ++j) yl[q][j] = a.Y[(r - s) * a.ldy + j];
        }
      }
    }
    const double dg = a.coef[r];
    double ky[KP];
#pragma unroll
    for (int j = 0; j < KP; ++j) {
      double v = dg * y[j];
#pragma unroll
      for (int q = 0; q < 3; ++q) v = fma(up[q], yu[q][j], fma(lo[q], yl[q][j], v));
      ky[j] = v;
    }
    const double bv = a.b ? a.b[r] : 0.0;
#pragma unroll
    for (int c = 0; c < KP; ++c) {
      double v = 0.0;
#pragma unroll
      for (int j = 0; j < KP; ++j) v = fma(y[j], a1[c][j], fma(ky[j], a2[c][j], v));
      if (a.b) v -= bv * rs[c];
      if (b0[c] >= 0) v -= a.B0[r * a.ldb0 + b0[c]];
      a.R[r * a.ldr + c] = v;
      nacc[c] = fma(v, v, nacc[c]);
    }
  }
  // fixed-order fold: lanes of a wavefront, then the 4 wavefronts
#pragma unroll
  for (int off = 1; off < 64; off <<= 1)
#pragma unroll
    for (int c = 0; c < KP; ++c) nacc[c] += __shfl_xor(nacc[c], off);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  if (l == 0) {
#pragma unroll
    for (int c = 0; c < KP; ++c) red[w * KP + c] = nacc[c];
  }
  __syncthreads();
  if (threadIdx.x < KP)
    a.partials[(int64_t)threadIdx.x * gridDim.x + blockIdx.x] =
        ((red[threadIdx.x] + red[KP + threadIdx.x]) + red[2 * KP + threadIdx.x]) + red[3 * KP + threadIdx.x];
}

template <int KP>
void launch_res(bkts_ctx ctx, const bkts_op_s& op, ResArgs a, double* nrm) {
  using G = TileGeom<KP>;
  const int64_t ntiles = (a.N + G::RT - 1) / G::RT;
  const int64_t cap = 3 * (int64_t)ctx->num_cu;  // the LDS tile pair admits 3 workgroups per CU at k = 4
  int64_t ns = ntiles < cap ? ntiles : cap;
  if (ns < 1) ns = 1;
  a.tps = (ntiles + ns - 1) / ns;
  a.partials = ctx->ws.get<double>("res_partials", (size_t)KP * ns);
  const double mat = op.st_na > 0 ? 8.0 * (1 + op.st_na) * op.N : op.nnz * 12.0 + 4.0 * (op.N + 1);
  ProfScope prof(ctx, BKTS_K_RESIDUAL, mat + 16.0 * op.N * a.k + (a.b ? 8.0 * op.N : 0.0) + 8.0 * op.N * a.nb0);
  if (op.st_na > 0 && KP <= 4 && a.k == KP) {
    int64_t nr = (a.N + 255) / 256;
    const int64_t rcap = 4 * (int64_t)ctx->num_cu;
    if (nr > rcap) nr = rcap;
    if (nr < 1) nr = 1;
    a.partials = ctx->ws.get<double>("res_partials", (size_t)KP * nr);
    launch(ctx, (st_residual_row_kernel<KP>), dim3(nr), dim3(256), 0, a);
    ns = nr;
  } else if (op.st_na > 0)
    launch(ctx, (residual_kernel<KP, 2>), dim3(ns), dim3(256), 0, a);
  else if (op.format == BKTS_FMT_SELL)
    launch(ctx, (residual_kernel<KP, 1>), dim3(ns), dim3(256), 0, a);
  else
    launch(ctx, (residual_kernel<KP, 0>), dim3(ns), dim3(256), 0, a);
  BKTS_HIP(hipGetLastError());
  prof.end();
  finalize_partials(ctx, a.partials, (int)ns, a.k, nrm);
}

}  // namespace

void residual(bkts_ctx ctx, const bkts_op_s& op, int k, const double* Y, int ldy, const double* A1t,
              const double* A2t, const double* b_rowsum, const double* B0, int ldb0, int nb0, const int* b0_to_col,
              double* R, int ldr, double* nrm) {
  BKTS_REQUIRE(nb0 >= 0 && nb0 <= kMaxB0, "at most %d B0 columns", kMaxB0);
  ResArgs a{};
  a.N = op.N;
  a.k = k;
  a.rowptr = op.rowptr.as<int32_t>();
  const bool sell = op.format == BKTS_FMT_SELL;
  a.col = sell ? op.sell_col.as<int32_t>() : op.col.as<int32_t>();
  a.val = sell ? op.sell_val.as<double>() : op.val.as<double>();
  a.sptr = op.sell_ptr.as<int64_t>();
  a.sw = op.sell_w.as<int32_t>();
  a.C = op.sell_C;
  a.uw = op.sell_uniform_w;
  a.na = op.st_na;
  for (int q = 0; q < 3; ++q) a.soff[q] = op.st_off[q];
  a.coef = op.st_coef.as<double>();
  a.Y = Y;
  a.ldy = ldy;
  a.A1 = A1t;
  a.A2 = A2t;
  a.b = op.b_nonzero ? op.b.as<double>() : nullptr;
  a.rs = b_rowsum;
  a.B0 = B0;
  a.ldb0 = ldb0;
  a.nb0 = B0 ? nb0 : 0;
  for (int j = 0; j < kMaxB0; ++j) a.b0col[j] = j < a.nb0 ? b0_to_col[j] : -1;
  a.R = R;
  a.ldr = ldr;
  switch (k <= 1 ? 1 : k <= 2 ? 2 : k <= 4 ? 4 : k <= 8 ? 8 : k <= 16 ? 16 : 32) {
    case 1: launch_res<1>(ctx, op, a, nrm); break;
    case 2: launch_res<2>(ctx, op, a, nrm); break;
    case 4: launch_res<4>(ctx, op, a, nrm); break;
    case 8: launch_res<8>(ctx, op, a, nrm); break;
    case 16: launch_res<16>(ctx, op, a, nrm); break;
    default: launch_res<32>(ctx, op, a, nrm); break;
  }
}

}  // namespace bkts

// Operator setup on the device: cell-centred FV assembly of K and b, CSR import, the SELL-C copy
// used by the block operator, the diagonal used by Jacobi, and the FP32 value copies.
#include "devcommon.hpp"
#include "internal.hpp"

namespace bkts {
namespace {

constexpr int kScanItems = 8;
constexpr int kScanTile = dev::kThreads * kScanItems;

// Exclusive scan of int64 counts in tiles of kScanTile: local scan + tile totals.
__global__ __launch_bounds__(256) void scan_tiles(const int64_t* in, int64_t n, int64_t* out, int64_t* totals) {
  __shared__ int64_t s[dev::kThreads];
  const int t = threadIdx.x;
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)t * kScanItems;
  int64_t v[kScanItems];
  int64_t run = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    v[i] = (base + i < n) ? in[base + i] : 0;
    run += v[i];
  }
  s[t] = run;
  __syncthreads();
  for (int off = 1; off < dev::kThreads; off <<= 1) {  // Hillis-Steele inclusive scan of thread sums
    int64_t add = (t >= off) ? s[t - off] : 0;
    __syncthreads();
    s[t] += add;
    __syncthreads();
  }
  int64_t acc = s[t] - run;  // exclusive prefix of this thread
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    if (base + i < n) out[base + i] = acc;
    acc += v[i];
  }
  if (t == dev::kThreads - 1) totals[blockIdx.x] = s[t];
}

// Sequential exclusive scan of the tile totals by one workgroup (chunks of 256, in order).
__global__ __launch_bounds__(256) void scan_totals(int64_t* totals, int64_t ntiles, int64_t* grand) {
  __shared__ int64_t s[dev::kThreads];
  __shared__ int64_t carry;
  const int t = threadIdx.x;
  if (t == 0) carry = 0;
  __syncthreads();
  for (int64_t c0 = 0; c0 < ntiles; c0 += dev::kThreads) {
    int64_t v = (c0 + t < ntiles) ? totals[c0 + t] : 0;
    s[t] = v;
    __syncthreads();
    for (int off = 1; off < dev::kThreads; off <<= 1) {
      int64_t add = (t >= off) ? s[t - off] : 0;
      __syncthreads();
      s[t] += add;
      __syncthreads();
    }
    if (c0 + t < ntiles) totals[c0 + t] = carry + s[t] - v;
    __syncthreads();
    if (t == dev::kThreads - 1) carry += s[t];
    __syncthreads();
  }
  if (t == 0) *grand = carry;
}

__global__ void scan_add(int64_t* out, int64_t n, const int64_t* totals) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] += totals[i / kScanTile];
}

// Exclusive scan of n counts into out[0..n]; out[n] = total.  Returns total (synchronises).
int64_t device_exclusive_scan(bkts_ctx ctx, const int64_t* in, int64_t n, int64_t* out) {
  const int64_t ntiles = (n + kScanTile - 1) / kScanTile;
  int64_t* totals = ctx->ws.get<int64_t>("scan_totals", ntiles + 1);
  if (n > 0) {
    launch(ctx, scan_tiles, dim3(ntiles), dim3(256), 0, in, n, out, totals);
    launch(ctx, scan_totals, dim3(1), dim3(256), 0, totals, ntiles, out + n);
    launch(ctx, scan_add, dim3((n + 255) / 256), dim3(256), 0, out, n, totals);
  } else {
    BKTS_HIP(hipMemsetAsync(out, 0, sizeof(int64_t), ctx->stream));
  }
  BKTS_HIP(hipGetLastError());
  int64_t total = 0;
  BKTS_HIP(hipMemcpyAsync(&total, out + n, sizeof(int64_t), hipMemcpyDeviceToHost, ctx->stream));
  ctx->sync();
  return total;
}

struct GridDev {
  int dim;
  int n[3];
  double h[3];
};

struct FvDev {
  const double* kappa;
  double kappa_const;
  double vel[3];
  int bc_type[6];
  double bc_val[6];
};

__device__ __forceinline__ void cell_coords(const GridDev& g, int64_t r, int (&i)[3]) {
  int64_t q = r;
  for (int d = 0; d < 3; ++d) {
    if (d < g.dim) {
      i[d] = (int)(q % g.n[d]);
      q /= g.n[d];
    } else {
      i[d] = 0;
    }
  }
}

__device__ __forceinline__ int64_t axis_stride(const GridDev& g, int d) {
  int64_t s = 1;
  for (int e = 0; e < d; ++e) s *= g.n[e];
  return s;
}

__global__ void fv_row_lengths(GridDev g, int64_t N, int64_t* len) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= N) return;
  int i[3];
  cell_coords(g, r, i);
  int64_t m = 1;
  for (int d = 0; d < g.dim; ++d) m += (i[d] > 0) + (i[d] < g.n[d] - 1);
  len[r] = m;
}

__device__ __forceinline__ double kap_at(const FvDev& c, int64_t r) {
  return c.kappa ? c.kappa[r] : c.kappa_const;
}

// One thread per cell: writes the row's entries in increasing column order
// (z-, y-, x-, diagonal, x+, y+, z+) and the cell's source term.
__global__ void fv_fill(GridDev g, FvDev c, int64_t N, const int64_t* rowptr64, int32_t* rowptr,
                        int32_t* col, double* val, double* b) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= N) return;
  int i[3];
  cell_coords(g, r, i);
  const double kP = kap_at(c, r);
  double diag = 0.0, src = 0.0;
  double offv[6];
  int64_t offc[6];
  bool has[6];
  for (int f = 0; f < 6; ++f) has[f] = false;
  for (int d = 0; d < g.dim; ++d) {
    const double h = g.h[d];
    const int64_t st = axis_stride(g, d);
    for (int side = 0; side < 2; ++side) {
      const int f = 2 * d + side;
      const bool interior = side == 0 ? (i[d] > 0) : (i[d] < g.n[d] - 1);
      const double w_out = side == 0 ? -c.vel[d] : c.vel[d];  // outward normal velocity
      if (interior) {
        const int64_t q = side == 0 ? r - st : r + st;
        const double kQ = kap_at(c, q);
        const double ks = kP + kQ;
        const double kf = ks > 0.0 ? 2.0 * kP * kQ / ks : 0.0;
        const double t = kf / (h * h);
        double off = -t;
        diag += t;
        if (w_out > 0.0) diag += w_out / h;       // outflow: upwind value is u_P
        else if (w_out < 0.0) off += w_out / h;   // inflow: upwind value is u_Q
        has[f] = true;
        offv[f] = off;
        offc[f] = q;
      } else if (c.bc_type[f] == BKTS_BC_DIRICHLET) {
        const double g_ = c.bc_val[f];
        const double tb = 2.0 * kP / (h * h);
        diag += tb;
        src += tb * g_;
        if (w_out > 0.0) diag += w_out / h;
        else if (w_out < 0.0) src -= w_out * g_ / h;
      }
    }
  }
  int64_t p = rowptr64[r];
  rowptr[r] = (int32_t)p;
  if (r == N - 1) rowptr[N] = (int32_t)rowptr64[N];
  for (int d = g.dim - 1; d >= 0; --d) {  // lower neighbours, farthest first
    const int f = 2 * d;
    if (has[f]) { col[p] = (int32_t)offc[f]; val[p] = offv[f]; ++p; }
  }
  col[p] = (int32_t)r;
  val[p] = diag;
  ++p;
  for (int d = 0; d < g.dim; ++d) {  // upper neighbours, nearest first
    const int f = 2 * d + 1;
    if (has[f]) { col[p] = (int32_t)offc[f]; val[p] = offv[f]; ++p; }
  }
  b[r] = src;
}

__global__ void csr_diag(int64_t N, const int32_t* rowptr, const int32_t* col, const double* val, double* diag) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= N) return;
  double d = 0.0;
  for (int32_t j = rowptr[r]; j < rowptr[r + 1]; ++j)
    if (col[j] == r) d += val[j];
  diag[r] = d;
}

__global__ void to_f32(int64_t n, const double* in, float* out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = (float)in[i];
}

__global__ void sell_widths(int64_t N, int C, int64_t nslices, const int32_t* rowptr, int64_t* wC, int32_t* w) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nslices) return;
  int32_t m = 0;
  for (int64_t r = s * C; r < (s + 1) * C && r < N; ++r) {
    int32_t l = rowptr[r + 1] - rowptr[r];
    m = l > m ? l : m;
  }
  w[s] = m;
  wC[s] = (int64_t)m * C;
}

__global__ void sell_fill(int64_t N, int C, const int32_t* rowptr, const int32_t* col, const double* val,
                          const int64_t* sptr, const int32_t* w, int32_t* scol, double* sval) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t s = r / C;
  const int64_t nslot_rows = ((N + C - 1) / C) * C;
  if (r >= nslot_rows) return;
  const int lr = (int)(r - s * C);
  const int ws = w[s];
  const int64_t base = sptr[s] + lr;
  int j = 0;
  if (r < N) {
    for (int32_t e = rowptr[r]; e < rowptr[r + 1]; ++e, ++j) {
      scol[base + (int64_t)j * C] = col[e];
      sval[base + (int64_t)j * C] = val[e];
    }
  }
  const int32_t pad_col = (int32_t)(r < N ? r : N - 1);
  for (; j < ws; ++j) {
    scol[base + (int64_t)j * C] = pad_col;
    sval[base + (int64_t)j * C] = 0.0;
  }
}

}  // namespace

void op_build_sell(bkts_op op) {
  bkts_ctx ctx = op->ctx;
  const int C = op->sell_C;
  const int64_t N = op->N;
  op->nslices = (N + C - 1) / C;
  DevBuf wC;
  wC.alloc(sizeof(int64_t) * (op->nslices + 1));
  op->sell_w.alloc(sizeof(int32_t) * op->nslices);
  op->sell_ptr.alloc(sizeof(int64_t) * (op->nslices + 1));
  launch(ctx, sell_widths, dim3((op->nslices + 255) / 256), dim3(256), 0, N, C, op->nslices,
                     op->rowptr.as<int32_t>(), wC.as<int64_t>(), op->sell_w.as<int32_t>());
  BKTS_HIP(hipGetLastError());
  // Uniform slice width when padding every slice to the widest costs at most 5%: the block operator
  // then derives slice offsets arithmetically instead of loading them.
  {
    std::vector<int32_t> hw(op->nslices);
    BKTS_HIP(hipMemcpyAsync(hw.data(), op->sell_w.p, sizeof(int32_t) * op->nslices, hipMemcpyDeviceToHost, ctx->stream));
    ctx->sync();
    int64_t sum = 0;
    int32_t wmax = 0;
    for (int32_t w : hw) {
      sum += w;
      wmax = w > wmax ? w : wmax;
    }
    if (wmax > 0 && (double)wmax * op->nslices <= 1.05 * (double)sum) {
      op->sell_uniform_w = wmax;
      std::vector<int64_t> hwc(op->nslices, (int64_t)wmax * C);
      for (auto& w : hw) w = wmax;
      BKTS_HIP(hipMemcpyAsync(op->sell_w.p, hw.data(), sizeof(int32_t) * op->nslices, hipMemcpyHostToDevice, ctx->stream));
      BKTS_HIP(hipMemcpyAsync(wC.p, hwc.data(), sizeof(int64_t) * op->nslices, hipMemcpyHostToDevice, ctx->stream));
      ctx->sync();
    }
  }
  op->sell_nnz = device_exclusive_scan(ctx, wC.as<int64_t>(), op->nslices, op->sell_ptr.as<int64_t>());
  BKTS_REQUIRE(op->sell_nnz < (int64_t)1 << 31, "SELL storage exceeds int32 indexing");
  op->sell_col.alloc(sizeof(int32_t) * op->sell_nnz);
  op->sell_val.alloc(sizeof(double) * op->sell_nnz);
  op->sell_val32.alloc(sizeof(float) * op->sell_nnz);
  const int64_t rows = op->nslices * C;
  if (op->sell_nnz > 0)
    launch(ctx, sell_fill, dim3((rows + 255) / 256), dim3(256), 0, N, C, op->rowptr.as<int32_t>(),
                     op->col.as<int32_t>(), op->val.as<double>(), op->sell_ptr.as<int64_t>(),
                     op->sell_w.as<int32_t>(), op->sell_col.as<int32_t>(), op->sell_val.as<double>());
  if (op->sell_nnz > 0)
    launch(ctx, to_f32, dim3((op->sell_nnz + 255) / 256), dim3(256), 0, op->sell_nnz,
                       op->sell_val.as<double>(), op->sell_val32.as<float>());
  BKTS_HIP(hipGetLastError());
}

void op_refresh_values(bkts_op op) {
  bkts_ctx ctx = op->ctx;
  const int64_t N = op->N;
  launch(ctx, csr_diag, dim3((N + 255) / 256), dim3(256), 0, N, op->rowptr.as<int32_t>(),
                     op->col.as<int32_t>(), op->val.as<double>(), op->diag.as<double>());
  if (op->nnz > 0)
    launch(ctx, to_f32, dim3((op->nnz + 255) / 256), dim3(256), 0, op->nnz,
                       op->val.as<double>(), op->val32.as<float>());
  if (op->format == BKTS_FMT_SELL && op->sell_nnz > 0) {
    const int64_t rows = op->nslices * op->sell_C;
    launch(ctx, sell_fill, dim3((rows + 255) / 256), dim3(256), 0, N, op->sell_C,
                       op->rowptr.as<int32_t>(), op->col.as<int32_t>(), op->val.as<double>(),
                       op->sell_ptr.as<int64_t>(), op->sell_w.as<int32_t>(), op->sell_col.as<int32_t>(),
                       op->sell_val.as<double>());
    launch(ctx, to_f32, dim3((op->sell_nnz + 255) / 256), dim3(256), 0, op->sell_nnz,
                       op->sell_val.as<double>(), op->sell_val32.as<float>());
  }
  BKTS_HIP(hipGetLastError());
}

void op_finish(bkts_op op) {
  bkts_ctx ctx = op->ctx;
  const int64_t N = op->N;
  op->diag.alloc(sizeof(double) * N);
  launch(ctx, csr_diag, dim3((N + 255) / 256), dim3(256), 0, N, op->rowptr.as<int32_t>(),
                     op->col.as<int32_t>(), op->val.as<double>(), op->diag.as<double>());
  op->val32.alloc(sizeof(float) * (op->nnz > 0 ? op->nnz : 1));
  if (op->nnz > 0)
    launch(ctx, to_f32, dim3((op->nnz + 255) / 256), dim3(256), 0, op->nnz,
                       op->val.as<double>(), op->val32.as<float>());
  BKTS_HIP(hipGetLastError());
  if (op->format == BKTS_FMT_SELL) op_build_sell(op);
  ctx->sync();
}

bkts_op fv_assemble(bkts_ctx ctx, const bkts_grid* grid, const bkts_fv_coeffs* c, int format) {
  BKTS_REQUIRE(grid && c, "grid and coeffs must not be NULL");
  BKTS_REQUIRE(grid->dim >= 1 && grid->dim <= 3, "grid dim must be 1, 2 or 3 (got %d)", grid->dim);
  BKTS_REQUIRE(format == BKTS_FMT_CSR || format == BKTS_FMT_SELL || format == BKTS_FMT_STENCIL,
               "unknown format %d", format);
  GridDev g{};
  g.dim = grid->dim;
  int64_t N = 1;
  for (int d = 0; d < 3; ++d) {
    if (d < grid->dim) {
      BKTS_REQUIRE(grid->n[d] >= 1, "grid n[%d] must be >= 1", d);
      g.n[d] = grid->n[d];
      g.h[d] = 1.0 / grid->n[d];
      N *= grid->n[d];
    } else {
      g.n[d] = 1;
      g.h[d] = 1.0;
    }
  }
  BKTS_REQUIRE(N * (2 * grid->dim + 1) < ((int64_t)1 << 31), "grid too large for int32 CSR indices");
  for (int f = 0; f < 6; ++f)
    BKTS_REQUIRE(c->bc_type[f] == BKTS_BC_DIRICHLET || c->bc_type[f] == BKTS_BC_NEUMANN, "bad bc_type[%d]", f);
  FvDev fd{};
  fd.kappa = c->kappa;
  fd.kappa_const = c->kappa_const;
  for (int d = 0; d < 3; ++d) fd.vel[d] = d < grid->dim ? c->velocity[d] : 0.0;
  for (int f = 0; f < 6; ++f) {
    fd.bc_type[f] = c->bc_type[f];
    fd.bc_val[f] = c->bc_value[f];
  }
  bkts_op op = new bkts_op_s();
  try {
    op->ctx = ctx;
    op->N = N;
    op->format = format == BKTS_FMT_STENCIL ? BKTS_FMT_SELL : format;  // SELL serves the other kernels
    op->grid = *grid;
    DevBuf len, rp64;
    len.alloc(sizeof(int64_t) * N);
    rp64.alloc(sizeof(int64_t) * (N + 1));
    launch(ctx, fv_row_lengths, dim3((N + 255) / 256), dim3(256), 0, g, N, len.as<int64_t>());
    BKTS_HIP(hipGetLastError());
    op->nnz = device_exclusive_scan(ctx, len.as<int64_t>(), N, rp64.as<int64_t>());
    op->rowptr.alloc(sizeof(int32_t) * (N + 1));
    op->col.alloc(sizeof(int32_t) * op->nnz);
    op->val.alloc(sizeof(double) * op->nnz);
    op->b.alloc(sizeof(double) * N);
    launch(ctx, fv_fill, dim3((N + 255) / 256), dim3(256), 0, g, fd, N, rp64.as<int64_t>(),
                       op->rowptr.as<int32_t>(), op->col.as<int32_t>(), op->val.as<double>(), op->b.as<double>());
    BKTS_HIP(hipGetLastError());
    bool nz = false;
    for (int f = 0; f < 2 * grid->dim; ++f)
      if (c->bc_type[f] == BKTS_BC_DIRICHLET && c->bc_value[f] != 0.0) nz = true;
    op->b_nonzero = nz;
    op->strip_period = grid->dim == 3 ? (int64_t)g.n[0] * g.n[1] : grid->dim == 2 ? g.n[0] : 0;
    op_finish(op);
    if (format == BKTS_FMT_STENCIL) op_build_stencil(op);
  } catch (...) {
    delete op;
    throw;
  }
  return op;
}

__global__ void rowptr_to64(int64_t N, const int32_t* rp, int64_t* out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i <= N) out[i] = rp[i];
}

bkts_op op_from_csr(bkts_ctx ctx, int64_t N, int64_t nnz, const int32_t* rowptr, const int32_t* col,
                    const double* val, int format) {
  BKTS_REQUIRE(N >= 1 && nnz >= 0, "N must be >= 1 and nnz >= 0");
  BKTS_REQUIRE(rowptr && (nnz == 0 || (col && val)), "CSR pointers must not be NULL");
  BKTS_REQUIRE(format != BKTS_FMT_STENCIL, "the stencil format needs the grid of bkts_fv_assemble");
  BKTS_REQUIRE(format == BKTS_FMT_CSR || format == BKTS_FMT_SELL, "unknown format %d", format);
  BKTS_REQUIRE(nnz < ((int64_t)1 << 31) && N < ((int64_t)1 << 31), "CSR too large for int32 indices");
  // validate the row pointer on the host (one copy of N+1 ints): monotone, starts at 0, ends at nnz
  std::vector<int32_t> hrp(N + 1);
  BKTS_HIP(hipMemcpyAsync(hrp.data(), rowptr, sizeof(int32_t) * (N + 1), hipMemcpyDeviceToHost, ctx->stream));
  ctx->sync();
  BKTS_REQUIRE(hrp[0] == 0 && hrp[N] == nnz, "rowptr must start at 0 and end at nnz");
  for (int64_t r = 0; r < N; ++r) BKTS_REQUIRE(hrp[r] <= hrp[r + 1], "rowptr not monotone at row %lld", (long long)r);
  std::vector<int32_t> hcol(nnz);
  if (nnz) {
    BKTS_HIP(hipMemcpyAsync(hcol.data(), col, sizeof(int32_t) * nnz, hipMemcpyDeviceToHost, ctx->stream));
    ctx->sync();
    for (int64_t e = 0; e < nnz; ++e)
      BKTS_REQUIRE(hcol[e] >= 0 && hcol[e] < N, "column index out of range at entry %lld", (long long)e);
  }
  bkts_op op = new bkts_op_s();
  try {
    op->ctx = ctx;
    op->N = N;
    op->nnz = nnz;
    op->format = format;
    op->rowptr.alloc(sizeof(int32_t) * (N + 1));
    op->col.alloc(sizeof(int32_t) * (nnz > 0 ? nnz : 1));
    op->val.alloc(sizeof(double) * (nnz > 0 ? nnz : 1));
    op->b.alloc(sizeof(double) * N);
    BKTS_HIP(hipMemcpyAsync(op->rowptr.p, rowptr, sizeof(int32_t) * (N + 1), hipMemcpyDeviceToDevice, ctx->stream));
    if (nnz) {
      BKTS_HIP(hipMemcpyAsync(op->col.p, col, sizeof(int32_t) * nnz, hipMemcpyDeviceToDevice, ctx->stream));
      BKTS_HIP(hipMemcpyAsync(op->val.p, val, sizeof(double) * nnz, hipMemcpyDeviceToDevice, ctx->stream));
    }
    BKTS_HIP(hipMemsetAsync(op->b.p, 0, sizeof(double) * N, ctx->stream));
    op_finish(op);
  } catch (...) {
    delete op;
    throw;
  }
  return op;
}

}  // namespace bkts

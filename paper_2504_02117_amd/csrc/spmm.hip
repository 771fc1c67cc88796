// Block operator Y = cb*B + alpha*X + beta*K X for row-major N x k blocks (Sec. 3, "BOP").
//
// Each row of K is handled by LPR = KP/VEC lanes of one wave64; every lane owns VEC consecutive
// columns.  The LPR lanes of a row read the same matrix entry (one memory transaction per wave
// instruction), so each value/index pair streams from HBM once per block of k columns, while the
// X rows of the neighbours are read as contiguous k-element segments.  SELL-C (C = 64, sigma = 1)
// stores the entries slice-column-major so that the row groups of a wave read consecutive
// addresses; CSR is the general fallback.  Workgroups are remapped so that each XCD streams one
// contiguous row range, which keeps the X rows of nearby stencil neighbours in that XCD's L2.
#include "devcommon.hpp"
#include "internal.hpp"

namespace bkts {
namespace {

template <typename T, int V>
struct Vec {
  T v[V];
};

template <typename T, int V>
__device__ __forceinline__ Vec<T, V> vload(const T* p) {
  Vec<T, V> r;
  if constexpr (V == 1) {
    r.v[0] = *p;
  } else if constexpr (sizeof(T) * V == 16) {
    if constexpr (sizeof(T) == 8) {
      const double2 q = *reinterpret_cast<const double2*>(p);
      r.v[0] = q.x;
      r.v[1] = q.y;
    } else {
      const float4 q = *reinterpret_cast<const float4*>(p);
      r.v[0] = q.x;
      r.v[1] = q.y;
      r.v[2] = q.z;
      r.v[3] = q.w;
    }
  } else if constexpr (sizeof(T) * V == 32) {  // two 16-byte loads
    const Vec<T, V / 2> lo = vload<T, V / 2>(p), hi = vload<T, V / 2>(p + V / 2);
#pragma unroll
    for (int i = 0; i < V / 2; ++i) {
      r.v[i] = lo.v[i];
      r.v[V / 2 + i] = hi.v[i];
    }
  } else {
#pragma unroll
    for (int i = 0; i < V; ++i) r.v[i] = p[i];
  }
  return r;
}

template <typename T, int V>
__device__ __forceinline__ void vstore(T* p, const Vec<T, V>& r) {
  if constexpr (V == 1) {
    *p = r.v[0];
  } else if constexpr (sizeof(T) * V == 16) {
    if constexpr (sizeof(T) == 8) {
      *reinterpret_cast<double2*>(p) = double2{r.v[0], r.v[1]};
    } else {
      *reinterpret_cast<float4*>(p) = float4{r.v[0], r.v[1], r.v[2], r.v[3]};
    }
  } else {
#pragma unroll
    for (int i = 0; i < V; ++i) p[i] = r.v[i];
  }
}

// Streaming store of the output rows: Y is not re-read by this kernel, so its lines are marked
// non-temporal and do not displace the X rows that later stencil neighbours read from L2.
template <typename T, int V>
__device__ __forceinline__ void vstore_nt(T* p, const Vec<T, V>& r) {
  if constexpr (sizeof(T) * V == 16) {
    if constexpr (sizeof(T) == 8) {
      typedef double d2 __attribute__((ext_vector_type(2)));
      const d2 q = {r.v[0], r.v[1]};
      __builtin_nontemporal_store(q, reinterpret_cast<d2*>(p));
    } else {
      typedef float f4 __attribute__((ext_vector_type(4)));
      const f4 q = {r.v[0], r.v[1], r.v[2], r.v[3]};
      __builtin_nontemporal_store(q, reinterpret_cast<f4*>(p));
    }
  } else if constexpr (sizeof(T) * V == 32) {  // two 16-byte stores
    Vec<T, V / 2> lo, hi;
#pragma unroll
    for (int i = 0; i < V / 2; ++i) {
      lo.v[i] = r.v[i];
      hi.v[i] = r.v[V / 2 + i];
    }
    vstore_nt<T, V / 2>(p, lo);
    vstore_nt<T, V / 2>(p + V / 2, hi);
  } else {
#pragma unroll
    for (int i = 0; i < V; ++i) __builtin_nontemporal_store(r.v[i], p + i);
  }
}

template <typename T>
struct SpmmArgs {
  int64_t N;
  int k;
  const int32_t* rowptr;  // CSR
  const int32_t* col;
  const T* val;
  const int64_t* sptr;    // SELL
  const int32_t* sw;
  int C;
  int uw;                 // uniform SELL width (0: load per-slice pointers)
  int64_t strip;          // > 0: XCD-strip schedule with this many blocks per strip
  T cb, alpha, beta;
  const T* B;
  int ldb;
  const T* X;
  int ldx;
  T* Y;
  int ldy;
};

constexpr int kUnroll = 8;

template <typename T, int KP, int VEC, bool SELL>
__global__ __launch_bounds__(256) void spmm_kernel(SpmmArgs<T> a) {
  constexpr int LPR = KP / VEC;
  constexpr int RPB = dev::kThreads / LPR;
  const int t = threadIdx.x;
  const int c0 = (t % LPR) * VEC;
  int64_t tile;
  if (a.strip > 0) {
    // XCD-strip schedule: XCD x (= dispatch index mod 8) takes strips x, x+8, x+16, ... in order, so
    // the rows one reuse period away are processed by the same XCD shortly before/after.
    const int64_t b = blockIdx.x, x = b % dev::kXcd, i = b / dev::kXcd;
    tile = ((i / a.strip) * dev::kXcd + x) * a.strip + i % a.strip;
  } else {
    tile = dev::xcd_slot(blockIdx.x, gridDim.x);
  }
  const int64_t r = tile * RPB + t / LPR;
  if (r >= a.N) return;
  const bool active = c0 < a.k;
  Vec<T, VEC> acc;
#pragma unroll
  for (int i = 0; i < VEC; ++i) acc.v[i] = T(0);

  int64_t base, stride, len;
  if constexpr (SELL) {
    const int64_t s = r / a.C;
    if (a.uw > 0) {
      base = s * a.C * a.uw + (r - s * a.C);
      len = a.uw;
    } else {
      base = a.sptr[s] + (r - s * a.C);
      len = a.sw[s];
    }
    stride = a.C;
  } else {
    base = a.rowptr[r];
    stride = 1;
    len = a.rowptr[r + 1] - base;
  }
  for (int64_t j0 = 0; j0 < len; j0 += kUnroll) {
    T v[kUnroll];
    int32_t cidx[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const bool ok = j0 + u < len;
      const int64_t e = base + (j0 + u) * stride;
      if constexpr (SELL) {  // coalesced single-use stream: non-temporal, keeps L2 for the X rows
        v[u] = ok ? __builtin_nontemporal_load(a.val + e) : T(0);
        cidx[u] = ok ? __builtin_nontemporal_load(a.col + e) : (int32_t)r;
      } else {
        v[u] = ok ? a.val[e] : T(0);
        cidx[u] = ok ? a.col[e] : (int32_t)r;
      }
    }
    if (active) {
      Vec<T, VEC> x[kUnroll];
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) x[u] = vload<T, VEC>(a.X + (int64_t)cidx[u] * a.ldx + c0);
#pragma unroll
      for (int u = 0; u < kUnroll; ++u)
#pragma unroll
        for (int i = 0; i < VEC; ++i) acc.v[i] = fma(v[u], x[u].v[i], acc.v[i]);
    }
  }
  if (!active) return;
  Vec<T, VEC> out;
  const Vec<T, VEC> xr = vload<T, VEC>(a.X + r * a.ldx + c0);
#pragma unroll
  for (int i = 0; i < VEC; ++i) out.v[i] = a.beta * acc.v[i] + a.alpha * xr.v[i];
  if (a.B) {
    const Vec<T, VEC> br = vload<T, VEC>(a.B + r * a.ldb + c0);
#pragma unroll
    for (int i = 0; i < VEC; ++i) out.v[i] = fma(a.cb, br.v[i], out.v[i]);
  }
  vstore<T, VEC>(a.Y + r * a.ldy + c0, out);
}

// Uniform-width SELL (every slice padded to the same width W <= 8, as for stencil operators):
// slice offsets are arithmetic and every thread carries G rows (RPB apart), so the matrix loads of
// all G rows are in flight before their dependent X-row loads, which are again all in flight
// before the first FMA.  Branch-free: padding entries and rows past N read a valid row with a
// zero weight.
template <typename T, int KP, int VEC, int G, bool NTS>
__global__ __launch_bounds__(256) void spmm_ell_kernel(SpmmArgs<T> a) {
  constexpr int LPR = KP / VEC;
  constexpr int RPB = dev::kThreads / LPR;
  const int t = threadIdx.x;
  const int c0 = (t % LPR) * VEC;
  int64_t tile;
  if (a.strip > 0) {
    const int64_t b = blockIdx.x, x = b % dev::kXcd, i = b / dev::kXcd;
    tile = ((i / a.strip) * dev::kXcd + x) * a.strip + i % a.strip;
  } else {
    tile = dev::xcd_slot(blockIdx.x, gridDim.x);
  }
  if (c0 >= a.k) return;
  const int W = a.uw;
  const int64_t nslot_rows = ((a.N + a.C - 1) / a.C) * a.C;  // rows covered by slices (padding rows exist)
  int64_t r[G];
  T v[G][kUnroll];
  int32_t ci[G][kUnroll];
#pragma unroll
  for (int g = 0; g < G; ++g) {
    r[g] = (tile * G + g) * RPB + t / LPR;
    const int64_t rs = r[g] < nslot_rows ? r[g] : nslot_rows - 1;
    const int64_t s = rs / a.C;
    const int64_t base = s * a.C * W + (rs - s * a.C);
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const int64_t e = base + (int64_t)(u < W ? u : W - 1) * a.C;
      v[g][u] = u < W ? __builtin_nontemporal_load(a.val + e) : T(0);
      ci[g][u] = __builtin_nontemporal_load(a.col + e);
    }
  }
  Vec<T, VEC> x[G][kUnroll];
#pragma unroll
  for (int g = 0; g < G; ++g)
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) x[g][u] = vload<T, VEC>(a.X + (int64_t)ci[g][u] * a.ldx + c0);
#pragma unroll
  for (int g = 0; g < G; ++g) {
    if (r[g] >= a.N) continue;
    Vec<T, VEC> acc;
#pragma unroll
    for (int i = 0; i < VEC; ++i) acc.v[i] = T(0);
#pragma unroll
    for (int u = 0; u < kUnroll; ++u)
#pragma unroll
      for (int i = 0; i < VEC; ++i) acc.v[i] = fma(v[g][u], x[g][u].v[i], acc.v[i]);
    const Vec<T, VEC> xr = vload<T, VEC>(a.X + r[g] * a.ldx + c0);
    Vec<T, VEC> out;
#pragma unroll
    for (int i = 0; i < VEC; ++i) out.v[i] = a.beta * acc.v[i] + a.alpha * xr.v[i];
    if (a.B) {
      const Vec<T, VEC> br = vload<T, VEC>(a.B + r[g] * a.ldb + c0);
#pragma unroll
      for (int i = 0; i < VEC; ++i) out.v[i] = fma(a.cb, br.v[i], out.v[i]);
    }
    if constexpr (NTS)
      vstore_nt<T, VEC>(a.Y + r[g] * a.ldy + c0, out);
    else
      vstore<T, VEC>(a.Y + r[g] * a.ldy + c0, out);
  }
}

// Uniform-width SELL with cooperative matrix loads, for wide rows (LPR = KP/VEC >= 2 lanes per
// row): lane l of a row's lane group loads entries l, l+LPR, ... of that row, and the entries are
// then broadcast inside the group with cross-lane shuffles.  One wave instruction thus fetches
// LPR entries of every row instead of one, which cuts the matrix-load instructions by LPR (the
// X-row gathers and the output store are as in the ELL kernel).  All lanes take part in the
// shuffles, so lanes past k (or rows past N) stay alive and only skip their X loads and stores.
template <typename T, int KP, int VEC>
__global__ __launch_bounds__(256) void spmm_coop_kernel(SpmmArgs<T> a) {
  constexpr int LPR = KP / VEC;
  constexpr int RPB = dev::kThreads / LPR;
  constexpr int NE = (kUnroll + LPR - 1) / LPR;  // entries per lane (W <= kUnroll)
  const int t = threadIdx.x;
  const int l = t % LPR, c0 = l * VEC;
  const int gb = (t & 63) & ~(LPR - 1);           // first lane of this row's group in the wave
  int64_t tile;
  if (a.strip > 0) {
    const int64_t b = blockIdx.x, x = b % dev::kXcd, i = b / dev::kXcd;
    tile = ((i / a.strip) * dev::kXcd + x) * a.strip + i % a.strip;
  } else {
    tile = dev::xcd_slot(blockIdx.x, gridDim.x);
  }
  const int W = a.uw;
  const int64_t nslot_rows = ((a.N + a.C - 1) / a.C) * a.C;
  const int64_t r = tile * RPB + t / LPR;
  const int64_t rs = r < nslot_rows ? r : nslot_rows - 1;
  const int64_t s = rs / a.C;
  const int64_t base = s * a.C * W + (rs - s * a.C);
  const int32_t self = (int32_t)(rs < a.N ? rs : a.N - 1);
  T vo[NE];
  int32_t co[NE];
#pragma unroll
  for (int e = 0; e < NE; ++e) {
    const int u = l + e * LPR;
    if (u < W) {
      vo[e] = __builtin_nontemporal_load(a.val + base + (int64_t)u * a.C);
      co[e] = __builtin_nontemporal_load(a.col + base + (int64_t)u * a.C);
    } else {
      vo[e] = T(0);
      co[e] = self;
    }
  }
  const bool active = c0 < a.k && r < a.N;
  Vec<T, VEC> acc;
#pragma unroll
  for (int i = 0; i < VEC; ++i) acc.v[i] = T(0);
  T v[kUnroll];
  Vec<T, VEC> x[kUnroll];
#pragma unroll
  for (int u = 0; u < kUnroll; ++u) {
    if (u < W) {  // uniform over the launch
      v[u] = __shfl(vo[u / LPR], gb + u % LPR, 64);
      const int32_t cu = __shfl(co[u / LPR], gb + u % LPR, 64);
      if (active) x[u] = vload<T, VEC>(a.X + (int64_t)cu * a.ldx + c0);
    }
  }
  if (!active) return;
#pragma unroll
  for (int u = 0; u < kUnroll; ++u) {
    if (u < W) {
#pragma unroll
      for (int i = 0; i < VEC; ++i) acc.v[i] = fma(v[u], x[u].v[i], acc.v[i]);
    }
  }
  const Vec<T, VEC> xr = vload<T, VEC>(a.X + r * a.ldx + c0);
  Vec<T, VEC> out;
#pragma unroll
  for (int i = 0; i < VEC; ++i) out.v[i] = a.beta * acc.v[i] + a.alpha * xr.v[i];
  if (a.B) {
    const Vec<T, VEC> br = vload<T, VEC>(a.B + r * a.ldb + c0);
#pragma unroll
    for (int i = 0; i < VEC; ++i) out.v[i] = fma(a.cb, br.v[i], out.v[i]);
  }
  vstore_nt<T, VEC>(a.Y + r * a.ldy + c0, out);
}

template <typename T, int KP, int VEC>
void launch_fmt(bkts_ctx ctx, const bkts_op_s& op, const SpmmArgs<T>& a) {
  constexpr int LPR = KP / VEC;
  // Uniform-width path, measured on the 128^3 7-point operator with cold inputs: rows of >= 16
  // bytes split over >= 2 lanes (FP64 k >= 8, FP32 k >= 16) take the cooperative-load kernel;
  // narrower rows the ELL kernel, with streaming stores from 8 columns on.  Two rows per thread
  // pay off only for narrow FP32 rows (FP64: registers).
  constexpr bool COOP = LPR >= 2 && KP * sizeof(T) >= 64;
  constexpr bool NTS = KP >= 8;
  constexpr int G = (sizeof(T) == 8 || KP >= 8) ? 1 : 2;
  const bool ell = op.format == BKTS_FMT_SELL && op.sell_uniform_w > 0 && op.sell_uniform_w <= kUnroll;
  const int RPB = dev::kThreads / LPR * (ell && !COOP ? G : 1);
  const int64_t ntiles = (a.N + RPB - 1) / RPB;
  int64_t nb = ntiles;
  SpmmArgs<T> aa = a;
  aa.strip = 0;
  if (op.strip_period >= (int64_t)dev::kXcd * RPB) {
    aa.strip = op.strip_period / dev::kXcd / RPB;
    const int64_t per = dev::kXcd * aa.strip;
    nb = (ntiles + per - 1) / per * per;  // whole rounds of 8 strips; blocks past the end exit
  }
  if (ell && COOP)
    launch(ctx, (spmm_coop_kernel<T, KP, VEC>), dim3(nb), dim3(dev::kThreads), 0, aa);
  else if (ell)
    launch(ctx, (spmm_ell_kernel<T, KP, VEC, G, NTS>), dim3(nb), dim3(dev::kThreads), 0, aa);
  else if (op.format == BKTS_FMT_SELL)
    launch(ctx, (spmm_kernel<T, KP, VEC, true>), dim3(nb), dim3(dev::kThreads), 0, aa);
  else
    launch(ctx, (spmm_kernel<T, KP, VEC, false>), dim3(nb), dim3(dev::kThreads), 0, aa);
}

template <typename T, int KP>
void launch_kp(bkts_ctx ctx, const bkts_op_s& op, const SpmmArgs<T>& a, bool vec_ok) {
  constexpr int VMAX = 16 / sizeof(T);
  if constexpr (KP >= VMAX) {
    if (vec_ok) {
      // Rows of 64 bytes or more on the uniform-width SELL path: 32 bytes per lane (two 16-byte
      // loads), half the lanes per row and twice the rows per workgroup.  On the 128^3 7-point
      // operator against 16 bytes per lane: FP64 k = 8 99 us (117), k = 16 181 us (201), k = 32
      // 363 us (435); FP32 k = 16 89 us (94), k = 32 154 us (187).  Rows of 32 bytes lose with it
      // (FP64 k = 4 69 us against 65.5, FP32 k = 8 55 us against 46).
      if constexpr (KP * sizeof(T) >= 64) {
        if (op.format == BKTS_FMT_SELL && op.sell_uniform_w > 0 && op.sell_uniform_w <= kUnroll)
          return launch_fmt<T, KP, 2 * VMAX>(ctx, op, a);
      }
      return launch_fmt<T, KP, VMAX>(ctx, op, a);
    }
  }
  launch_fmt<T, KP, 1>(ctx, op, a);
}

inline int padded_k(int k) {
  int kp = 1;
  while (kp < k) kp <<= 1;
  return kp;
}

template <typename T>
void spmm_t(bkts_ctx ctx, const bkts_op_s& op, int k, double cb, const void* B, int ldb, double alpha,
            const void* X, int ldx, double beta, void* Y, int ldy) {
  SpmmArgs<T> a{};
  a.N = op.N;
  a.k = k;
  a.rowptr = op.rowptr.as<int32_t>();
  const bool sell = op.format == BKTS_FMT_SELL;
  a.col = sell ? op.sell_col.as<int32_t>() : op.col.as<int32_t>();
  if constexpr (sizeof(T) == 8)
    a.val = sell ? op.sell_val.as<double>() : op.val.as<double>();
  else
    a.val = sell ? op.sell_val32.as<float>() : op.val32.as<float>();
  a.sptr = op.sell_ptr.as<int64_t>();
  a.sw = op.sell_w.as<int32_t>();
  a.C = op.sell_C;
  a.uw = op.sell_uniform_w;
  a.cb = (T)cb;
  a.alpha = (T)alpha;
  a.beta = (T)beta;
  a.B = static_cast<const T*>(B);
  a.ldb = ldb;
  a.X = static_cast<const T*>(X);
  a.ldx = ldx;
  a.Y = static_cast<T*>(Y);
  a.ldy = ldy;
  const int kp = padded_k(k);
  constexpr int VMAX = 16 / sizeof(T);
  const double sv = sizeof(T);
  ProfScope prof(ctx, BKTS_K_SPMM,
                 op.nnz * (sv + 4.0) + 4.0 * (op.N + 1) + (2.0 + (B ? 1.0 : 0.0)) * op.N * k * sv);
  auto aligned = [](const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; };
  const bool vec_ok = k == kp && ldx % VMAX == 0 && ldy % VMAX == 0 && aligned(X) && aligned(Y) &&
                      (!B || (ldb % VMAX == 0 && aligned(B)));
  switch (kp) {
    case 1: launch_kp<T, 1>(ctx, op, a, vec_ok); break;
    case 2: launch_kp<T, 2>(ctx, op, a, vec_ok); break;
    case 4: launch_kp<T, 4>(ctx, op, a, vec_ok); break;
    case 8: launch_kp<T, 8>(ctx, op, a, vec_ok); break;
    case 16: launch_kp<T, 16>(ctx, op, a, vec_ok); break;
    case 32: launch_kp<T, 32>(ctx, op, a, vec_ok); break;
    default: throw Error{BKTS_EINVAL, fmt("k=%d exceeds BKTS_MAX_K", k)};
  }
  BKTS_HIP(hipGetLastError());
}

}  // namespace

void spmm(bkts_ctx ctx, const bkts_op_s& op, int dtype, int k, double cb, const void* B, int ldb, double alpha,
          const void* X, int ldx, double beta, void* Y, int ldy) {
  if (op.N == 0) return;
  if (op.st_na > 0) return spmm_stencil(ctx, op, dtype, k, cb, B, ldb, alpha, X, ldx, beta, Y, ldy);
  if (dtype == BKTS_F64)
    spmm_t<double>(ctx, op, k, cb, B, ldb, alpha, X, ldx, beta, Y, ldy);
  else
    spmm_t<float>(ctx, op, k, cb, B, ldb, alpha, X, ldx, beta, Y, ldy);
}

}  // namespace bkts

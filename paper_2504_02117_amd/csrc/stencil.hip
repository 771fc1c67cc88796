// Index-free stencil form of the block operator (the BOP of Sec. 3 without its column-index
// stream) for symmetric 5/7-point operators on a structured grid, as produced by the cell-centred
// FV assembly without convection (Sec. 4.1).
//
// Rows are numbered ix + nx*iy + nx*ny*iz, so every off-diagonal entry sits at a fixed offset s_a
// in {1, nx, nx*ny}.  For a symmetric K the entry K[r, r + s_a] equals K[r + s_a, r], and one array
// per offset holds it once:  o_a[r] = K[r, r + s_a] (zero where r + s_a is not a neighbour: the
// + faces on the domain boundary).  With d[r] = K[r, r]
//
//   (K x)[r] = d[r] x[r] + sum_a ( o_a[r] x[r + s_a] + o_a[r - s_a] x[r - s_a] ).
//
// A neighbour index that wraps to the next grid line or plane meets a zero coefficient (o_a of a
// cell on the + boundary); only indices outside [0, N) are skipped.  The matrix stream drops from
// nnz * (value + index) bytes to (1 + dim) * N values: 4N against 14N words for the 7-point
// operator.  The arrays are extracted from the assembled CSR, which stays the operator's
// definition, and every entry is checked: an operator with an entry off the three offsets or a
// non-symmetric pair (convection) is rejected.
#include "devcommon.hpp"
#include "internal.hpp"

namespace bkts {
namespace {

struct StOff {
  int na;
  int64_t s[3];
};

// First offset index a with s_a == d (duplicated offsets, as for nx == 1, count once), or -1.
__device__ __forceinline__ int offset_index(const StOff& o, int64_t d) {
  for (int a = 0; a < o.na; ++a)
    if (o.s[a] == d) return a;
  return -1;
}

// d[r] and o_a[r] from the forward entries of row r; flags an entry at any other offset.
__global__ void st_fill(int64_t N, const int32_t* rowptr, const int32_t* col, const double* val, StOff o,
                        double* coef, int* bad) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= N) return;
  for (int32_t e = rowptr[r]; e < rowptr[r + 1]; ++e) {
    const int64_t c = col[e];
    const double v = val[e];
    if (c == r) {
      coef[r] += v;
      continue;
    }
    const int a = offset_index(o, c - r);
    if (a >= 0) {
      coef[(1 + a) * N + r] += v;
    } else if (offset_index(o, r - c) < 0 && v != 0.0) {
      atomicOr(bad, 1);
    }
  }
}

// Every backward entry K[r, r - s_a] must equal the forward one stored by row r - s_a (and be
// absent exactly when that one is zero).
__global__ void st_check(int64_t N, const int32_t* rowptr, const int32_t* col, const double* val, StOff o,
                         const double* coef, int* bad) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= N) return;
  for (int a = 0; a < o.na; ++a) {
    const int64_t c = r - o.s[a];
    double found = 0.0;
    for (int32_t e = rowptr[r]; e < rowptr[r + 1]; ++e)
      if (col[e] == c) found += val[e];
    const double want = c >= 0 ? coef[(1 + a) * N + c] : 0.0;
    if (found != want) atomicOr(bad, 2);
  }
}

__global__ void st_to_f32(int64_t n, const double* in, float* out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = (float)in[i];
}

template <typename T, int V>
struct SVec {
  T v[V];
};

template <typename T, int V>
__device__ __forceinline__ SVec<T, V> sload(const T* p) {
  SVec<T, V> r;
  if constexpr (sizeof(T) * V == 16 && sizeof(T) == 8) {
    const double2 q = *reinterpret_cast<const double2*>(p);
    r.v[0] = q.x;
    r.v[1] = q.y;
  } else if constexpr (sizeof(T) * V == 16) {
    const float4 q = *reinterpret_cast<const float4*>(p);
    r.v[0] = q.x;
    r.v[1] = q.y;
    r.v[2] = q.z;
    r.v[3] = q.w;
  } else {
#pragma unroll
    for (int i = 0; i < V; ++i) r.v[i] = p[i];
  }
  return r;
}

template <typename T, int V>
__device__ __forceinline__ void sstore(T* p, const SVec<T, V>& r, bool nt) {
  if constexpr (sizeof(T) * V == 16) {
    typedef T vt __attribute__((ext_vector_type(V)));
    vt q;
#pragma unroll
    for (int i = 0; i < V; ++i) q[i] = r.v[i];
    if (nt)
      __builtin_nontemporal_store(q, reinterpret_cast<vt*>(p));
    else
      *reinterpret_cast<vt*>(p) = q;
  } else {
#pragma unroll
    for (int i = 0; i < V; ++i) p[i] = r.v[i];
  }
}

template <typename T>
struct StArgs {
  int64_t N;
  int k;
  StOff o;
  const T* coef;  // (1 + na) arrays of N: d, o_0, ..., o_{na-1}
  int64_t strip;  // > 0: XCD-strip schedule with this many blocks per strip
  T cb, alpha, beta;
  const T* B;
  int ldb;
  const T* X;
  int ldx;
  T* Y;
  int ldy;
};

// Y = cb B + alpha X + beta K X.  Each row is handled by LPR = KP/VEC lanes, each owning VEC
// consecutive columns (16-byte accesses when the block allows); a thread carries G rows RPB apart,
// whose loads are all issued before the first FMA.  The diagonal stream is read non-temporally
// (single use); the o_a arrays are read twice (at r and at r - s_a, one line, one grid line or one
// plane later), so they stay cached for the second read.
template <typename T, int KP, int VEC, int G>
__global__ __launch_bounds__(256) void st_spmm_kernel(StArgs<T> a) {
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
  const int64_t N = a.N;
  int64_t r[G];
  T dg[G], up[G][3], lo[G][3];
  SVec<T, VEC> xr[G], xu[G][3], xl[G][3];
#pragma unroll
  for (int g = 0; g < G; ++g) {
    r[g] = (tile * G + g) * RPB + t / LPR;
    const bool ok = r[g] < N;
    dg[g] = ok ? __builtin_nontemporal_load(a.coef + r[g]) : T(0);
    if (ok) xr[g] = sload<T, VEC>(a.X + r[g] * a.ldx + c0);
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      up[g][q] = lo[g][q] = T(0);
      if (ok && q < a.o.na) {
        const int64_t s = a.o.s[q];
        const T* oq = a.coef + (1 + q) * N;
        if (r[g] + s < N) {
          up[g][q] = oq[r[g]];
          xu[g][q] = sload<T, VEC>(a.X + (r[g] + s) * a.ldx + c0);
        }
        if (r[g] - s >= 0) {
          lo[g][q] = oq[r[g] - s];
          xl[g][q] = sload<T, VEC>(a.X + (r[g] - s) * a.ldx + c0);
        }
      }
    }
  }
#pragma unroll
  for (int g = 0; g < G; ++g) {
    if (r[g] >= N) continue;
    SVec<T, VEC> acc;
#pragma unroll
    for (int i = 0; i < VEC; ++i) acc.v[i] = dg[g] * xr[g].v[i];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      if (q < a.o.na) {
        const int64_t s = a.o.s[q];
        if (r[g] - s >= 0) {
#pragma unroll
          for (int i = 0; i < VEC; ++i) acc.v[i] = fma(lo[g][q], xl[g][q].v[i], acc.v[i]);
        }
        if (r[g] + s < N) {
#pragma unroll
          for (int i = 0; i < VEC; ++i) acc.v[i] = fma(up[g][q], xu[g][q].v[i], acc.v[i]);
        }
      }
    }
    SVec<T, VEC> out;
#pragma unroll
    for (int i = 0; i < VEC; ++i) out.v[i] = a.beta * acc.v[i] + a.alpha * xr[g].v[i];
    if (a.B) {
      const SVec<T, VEC> br = sload<T, VEC>(a.B + r[g] * a.ldb + c0);
#pragma unroll
      for (int i = 0; i < VEC; ++i) out.v[i] = fma(a.cb, br.v[i], out.v[i]);
    }
    sstore<T, VEC>(a.Y + r[g] * a.ldy + c0, out, KP >= 8);
  }
}

// Wide rows on a 3-D grid (rows of 64 bytes or more: the SpMM is bound by gathering each row's six
// neighbours, not by HBM): a workgroup owns a TX x TY tile of grid columns and marches through a
// range of z-planes.  Three plane slots of (TX+2) x (TY+2) rows (the tile and its one-cell halo) rotate
// in LDS: each step loads plane z+1 once (coalesced 16-byte chunks, zeros outside the grid), stages
// the seven coefficients of plane z's tile rows once per row, and then every output chunk reads its
// row and its six neighbours from LDS.  Arithmetic order and the zero-coefficient rule are those of
// st_spmm_kernel (d x, then the lower and upper neighbour along x, y, z).  One-dimensional grid of
// tiles x z-chunks, remapped so that each XCD takes one contiguous range (neighbouring tiles, whose
// halos overlap, share that XCD's L2).
template <typename T>
struct StTileArgs {
  StArgs<T> s;
  int nx, ny, nz;
  int tiles_x, tiles_y, zlen;
};

template <typename T, int KP, int TX, int TY>
__global__ __launch_bounds__(256) void st_tile_kernel(StTileArgs<T> a) {
  constexpr int VEC = 16 / sizeof(T);
  constexpr int LPR = KP / VEC;  // 16-byte chunks per row
  constexpr int HX = TX + 2, HY = TY + 2, HP = HX * HY, TR = TX * TY;
  constexpr int PL = (HP * LPR + 255) / 256;  // plane chunks per thread
  constexpr int CL = (TR * 7 + 255) / 256;    // coefficients per thread
  typedef T vt __attribute__((ext_vector_type(VEC)));
  __shared__ vt xs[3][HP * LPR];
  __shared__ T cs[TR * 7];
  const int t = threadIdx.x;
  const int nx = a.nx, ny = a.ny, nz = a.nz;
  const int64_t plane = (int64_t)nx * ny, N = a.s.N;
  const int64_t ntile = (int64_t)a.tiles_x * a.tiles_y;
  const int64_t unit = dev::xcd_slot(blockIdx.x, gridDim.x);
  const int zc = (int)(unit / ntile), tile = (int)(unit - (int64_t)zc * ntile);
  const int tx0 = (tile % a.tiles_x) * TX, ty0 = (tile / a.tiles_x) * TY;
  const int z0 = zc * a.zlen;
  const int z1 = z0 + a.zlen < nz ? z0 + a.zlen : nz;
  const T* X = a.s.X;
  const int ldx = a.s.ldx;
  // All loads of a plane are issued before any of them is used: out-of-grid chunks read row 0 and
  // are replaced by zeros afterwards.
  auto fetch_plane = [&](int z, vt (&v)[PL]) {
#pragma unroll
    for (int i = 0; i < PL; ++i) {
      const int e = t + i * 256;
      const int row = e / LPR, c = e - row * LPR;
      const int hy = row / HX, hx = row - hy * HX;
      const int ix = tx0 - 1 + hx, iy = ty0 - 1 + hy;
      const bool ok = e < HP * LPR && z >= 0 && z < nz && ix >= 0 && ix < nx && iy >= 0 && iy < ny;
      const int64_t off = ok ? ((int64_t)z * plane + (int64_t)iy * nx + ix) * ldx + c * VEC : 0;
      v[i] = *reinterpret_cast<const vt*>(X + off);
      if (!ok) v[i] = (vt)(T(0));
    }
  };
  auto store_plane = [&](int slot, const vt (&v)[PL]) {
#pragma unroll
    for (int i = 0; i < PL; ++i) {
      const int e = t + i * 256;
      if (e < HP * LPR) xs[slot][e] = v[i];
    }
  };
  // coefficient q of a tile row: d; then the lower and the upper coupling along x, y, z (a lower
  // coupling across the grid boundary is zero)
  auto fetch_coef = [&](int z, T (&v)[CL]) {
#pragma unroll
    for (int i = 0; i < CL; ++i) {
      const int e = t + i * 256;
      const int row = e / 7, q = e - row * 7;
      const int ly = row / TX, lx = row - ly * TX;
      const int ix = tx0 + lx, iy = ty0 + ly;
      const int axis = (q + 1) >> 1;
      const bool lower = (q & 1) != 0;
      const int64_t st = axis == 1 ? 1 : (axis == 2 ? (int64_t)nx : plane);
      const bool inside = axis == 1 ? ix > 0 : (axis == 2 ? iy > 0 : z > 0);
      const bool ok = e < TR * 7 && z < nz && ix < nx && iy < ny && (!lower || inside);
      const int64_t r = (int64_t)z * plane + (int64_t)iy * nx + ix;
      const int64_t off = ok ? axis * N + r - (lower ? st : 0) : 0;
      v[i] = a.s.coef[off];
      if (!ok) v[i] = T(0);
    }
  };
  auto store_coef = [&](const T (&v)[CL]) {
#pragma unroll
    for (int i = 0; i < CL; ++i) {
      const int e = t + i * 256;
      if (e < TR * 7) cs[e] = v[i];
    }
  };
  if (z0 >= z1) return;
  // planes z-1, z, z+1 sit in the LDS slots while plane z+2 is in flight in registers and plane z+3
  // is being requested: two planes of loads in flight per workgroup
  vt pv[2][PL];
  T cv[2][CL];
  fetch_plane(z0 - 1, pv[0]);
  store_plane((z0 + 2) % 3, pv[0]);
  fetch_plane(z0, pv[0]);
  store_plane(z0 % 3, pv[0]);
  fetch_plane(z0 + 1, pv[0]);
  store_plane((z0 + 1) % 3, pv[0]);
  fetch_coef(z0, cv[0]);
  store_coef(cv[0]);
  if (z0 + 1 < z1) {
    fetch_plane(z0 + 2, pv[0]);
    fetch_coef(z0 + 1, cv[0]);
  }
  __syncthreads();
  for (int z = z0; z < z1; ++z) {
    const int b = (z - z0) & 1;
    if (z + 2 < z1) {
      fetch_plane(z + 3, pv[b ^ 1]);
      fetch_coef(z + 2, cv[b ^ 1]);
    }
    const vt* P0 = xs[z % 3];
    const vt* Pm = xs[(z + 2) % 3];
    const vt* Pp = xs[(z + 1) % 3];
    for (int e = t; e < TR * LPR; e += 256) {
      const int row = e / LPR, c = e - row * LPR;
      const int ly = row / TX, lx = row - ly * TX;
      const int ix = tx0 + lx, iy = ty0 + ly;
      if (ix >= nx || iy >= ny) continue;
      const int h = ((ly + 1) * HX + lx + 1) * LPR + c;
      const vt xc = P0[h];
      const T* cf = cs + row * 7;
      vt acc = cf[0] * xc;
      acc = __builtin_elementwise_fma((vt)cf[1], P0[h - LPR], acc);
      acc = __builtin_elementwise_fma((vt)cf[2], P0[h + LPR], acc);
      acc = __builtin_elementwise_fma((vt)cf[3], P0[h - HX * LPR], acc);
      acc = __builtin_elementwise_fma((vt)cf[4], P0[h + HX * LPR], acc);
      acc = __builtin_elementwise_fma((vt)cf[5], Pm[h], acc);
      acc = __builtin_elementwise_fma((vt)cf[6], Pp[h], acc);
      const int64_t r = (int64_t)z * plane + (int64_t)iy * nx + ix;
      vt out = a.s.beta * acc + a.s.alpha * xc;
      if (a.s.B) {
        const vt br = *reinterpret_cast<const vt*>(a.s.B + r * a.s.ldb + c * VEC);
        out = __builtin_elementwise_fma((vt)a.s.cb, br, out);
      }
      __builtin_nontemporal_store(out, reinterpret_cast<vt*>(a.s.Y + r * a.s.ldy + c * VEC));
    }
    __syncthreads();  // slot (z-1) % 3 and the coefficients are free
    if (z + 1 < z1) {
      store_plane((z + 2) % 3, pv[b]);
      store_coef(cv[b]);
    }
    __syncthreads();
  }
}

template <typename T, int KP, int TX, int TY>
void st_tile_launch(bkts_ctx ctx, const bkts_op_s& op, const StArgs<T>& s, int rounds) {
  StTileArgs<T> a;
  a.s = s;
  a.nx = op.grid.n[0];
  a.ny = op.grid.n[1];
  a.nz = op.grid.n[2];
  a.tiles_x = (a.nx + TX - 1) / TX;
  a.tiles_y = (a.ny + TY - 1) / TY;
  const int64_t ntile = (int64_t)a.tiles_x * a.tiles_y;
  // `rounds` rounds of resident workgroups (LDS bounds the occupancy); each z-chunk costs two extra
  // plane loads
  const int64_t resident =
      (int64_t)blocks_per_cu(reinterpret_cast<const void*>(st_tile_kernel<T, KP, TX, TY>)) * ctx->num_cu;
  int64_t nzc = (rounds * resident + ntile / 2) / ntile;
  if (nzc > a.nz) nzc = a.nz;
  if (nzc < 1) nzc = 1;
  a.zlen = (int)((a.nz + nzc - 1) / nzc);
  nzc = (a.nz + a.zlen - 1) / a.zlen;
  launch(ctx, (st_tile_kernel<T, KP, TX, TY>), dim3((unsigned)(ntile * nzc)), dim3(dev::kThreads), 0, a);
}

// Whether the tiled kernel serves this call: a 3-D grid with all three offsets, full-width 16-byte
// aligned blocks (vec_ok) and rows of 64 to 256 bytes.
template <typename T>
bool st_tile_fits(const bkts_op_s& op, int kp, bool vec_ok) {
  const int rowb = kp * (int)sizeof(T);
  return vec_ok && op.grid.dim == 3 && op.st_na == 3 && op.grid.n[0] >= 2 && op.grid.n[1] >= 2 &&
         op.grid.n[2] >= 2 && rowb >= 64 && rowb <= 256;
}

template <typename T, int KP, int VEC>
void st_launch(bkts_ctx ctx, const bkts_op_s& op, const StArgs<T>& a0) {
  constexpr int LPR = KP / VEC;
  // rows per thread: narrow rows carry several rows per thread (more loads in flight per wave)
  constexpr int G = KP * sizeof(T) <= 16 ? 2 : 1;
  constexpr int RPB = dev::kThreads / LPR * G;
  StArgs<T> a = a0;
  const int64_t ntiles = (a.N + RPB - 1) / RPB;
  int64_t nb = ntiles;
  a.strip = 0;
  if (op.strip_period >= (int64_t)dev::kXcd * RPB) {
    a.strip = op.strip_period / dev::kXcd / RPB;
    const int64_t per = dev::kXcd * a.strip;
    nb = (ntiles + per - 1) / per * per;  // whole rounds of 8 strips; blocks past the end exit
  }
  launch(ctx, (st_spmm_kernel<T, KP, VEC, G>), dim3(nb), dim3(dev::kThreads), 0, a);
}

template <typename T, int KP>
void st_launch_kp(bkts_ctx ctx, const bkts_op_s& op, const StArgs<T>& a, bool vec_ok) {
  constexpr int VMAX = 16 / sizeof(T);
  if constexpr (KP >= VMAX) {
    if (vec_ok) return st_launch<T, KP, VMAX>(ctx, op, a);
  }
  st_launch<T, KP, 1>(ctx, op, a);
}

template <typename T>
void st_spmm_t(bkts_ctx ctx, const bkts_op_s& op, int k, double cb, const void* B, int ldb, double alpha,
               const void* X, int ldx, double beta, void* Y, int ldy) {
  StArgs<T> a{};
  a.N = op.N;
  a.k = k;
  a.o.na = op.st_na;
  for (int q = 0; q < 3; ++q) a.o.s[q] = op.st_off[q];
  if constexpr (sizeof(T) == 8)
    a.coef = op.st_coef.as<double>();
  else
    a.coef = op.st_coef32.as<float>();
  a.cb = (T)cb;
  a.alpha = (T)alpha;
  a.beta = (T)beta;
  a.B = static_cast<const T*>(B);
  a.ldb = ldb;
  a.X = static_cast<const T*>(X);
  a.ldx = ldx;
  a.Y = static_cast<T*>(Y);
  a.ldy = ldy;
  int kp = 1;
  while (kp < k) kp <<= 1;
  constexpr int VMAX = 16 / sizeof(T);
  const double sv = sizeof(T);
  ProfScope prof(ctx, BKTS_K_SPMM, (1.0 + op.st_na) * op.N * sv + (2.0 + (B ? 1.0 : 0.0)) * op.N * k * sv);
  auto aligned = [](const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; };
  const bool vec_ok = k == kp && ldx % VMAX == 0 && ldy % VMAX == 0 && aligned(X) && aligned(Y) &&
                      (!B || (ldb % VMAX == 0 && aligned(B)));
  if (st_tile_fits<T>(op, kp, vec_ok)) {
    // tile shapes from a sweep on the 128^3 operator: the smaller the LDS footprint, the more
    // workgroups per CU keep loads in flight, which beats the larger halo share of a small tile
    if constexpr (sizeof(T) == 8) {
      if (kp == 8) st_tile_launch<T, 8, 16, 8>(ctx, op, a, 1);
      else if (kp == 16) st_tile_launch<T, 16, 8, 4>(ctx, op, a, 1);
      else st_tile_launch<T, 32, 8, 4>(ctx, op, a, 2);
    } else {
      if (kp == 16) st_tile_launch<T, 16, 16, 8>(ctx, op, a, 1);
      else st_tile_launch<T, 32, 8, 4>(ctx, op, a, 1);
    }
    BKTS_HIP(hipGetLastError());
    return;
  }
  switch (kp) {
    case 1: st_launch_kp<T, 1>(ctx, op, a, vec_ok); break;
    case 2: st_launch_kp<T, 2>(ctx, op, a, vec_ok); break;
    case 4: st_launch_kp<T, 4>(ctx, op, a, vec_ok); break;
    case 8: st_launch_kp<T, 8>(ctx, op, a, vec_ok); break;
    case 16: st_launch_kp<T, 16>(ctx, op, a, vec_ok); break;
    case 32: st_launch_kp<T, 32>(ctx, op, a, vec_ok); break;
    default: throw Error{BKTS_EINVAL, fmt("k=%d exceeds BKTS_MAX_K", k)};
  }
  BKTS_HIP(hipGetLastError());
}

}  // namespace

void op_build_stencil(bkts_op op) {
  bkts_ctx ctx = op->ctx;
  const bkts_grid& g = op->grid;
  BKTS_REQUIRE(g.dim >= 1 && g.dim <= 3, "the stencil form needs a structured grid");
  const int64_t N = op->N;
  StOff o{};
  int64_t stride = 1;
  for (int d = 0; d < g.dim; ++d) {
    bool dup = false;
    for (int q = 0; q < o.na; ++q) dup |= o.s[q] == stride;
    if (!dup && stride < N) o.s[o.na++] = stride;
    stride *= g.n[d];
  }
  op->st_na = 0;
  op->st_coef.alloc(sizeof(double) * (1 + o.na) * N);
  op->st_coef32.alloc(sizeof(float) * (1 + o.na) * N);
  int* bad = ctx->ws.get<int>("st_bad", 1);
  BKTS_HIP(hipMemsetAsync(op->st_coef.p, 0, sizeof(double) * (1 + o.na) * N, ctx->stream));
  BKTS_HIP(hipMemsetAsync(bad, 0, sizeof(int), ctx->stream));
  const dim3 grid((unsigned)((N + 255) / 256));
  launch(ctx, st_fill, grid, dim3(256), 0, N, op->rowptr.as<int32_t>(), op->col.as<int32_t>(),
         op->val.as<double>(), o, op->st_coef.as<double>(), bad);
  launch(ctx, st_check, grid, dim3(256), 0, N, op->rowptr.as<int32_t>(), op->col.as<int32_t>(),
         op->val.as<double>(), o, op->st_coef.as<double>(), bad);
  const int64_t n = (1 + o.na) * N;
  launch(ctx, st_to_f32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, n, op->st_coef.as<double>(),
         op->st_coef32.as<float>());
  BKTS_HIP(hipGetLastError());
  int hbad = 0;
  BKTS_HIP(hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
  ctx->sync();
  if (hbad) {
    op->st_coef.release();
    op->st_coef32.release();
    throw Error{BKTS_EINVAL, hbad & 1 ? "stencil format: an entry lies off the grid-neighbour offsets"
                                      : "stencil format needs a symmetric operator (no convection)"};
  }
  op->st_na = o.na;
  for (int q = 0; q < 3; ++q) op->st_off[q] = q < o.na ? o.s[q] : 0;
}

void spmm_stencil(bkts_ctx ctx, const bkts_op_s& op, int dtype, int k, double cb, const void* B, int ldb,
                  double alpha, const void* X, int ldx, double beta, void* Y, int ldy) {
  if (dtype == BKTS_F64)
    st_spmm_t<double>(ctx, op, k, cb, B, ldb, alpha, X, ldx, beta, Y, ldy);
  else
    st_spmm_t<float>(ctx, op, k, cb, B, ldb, alpha, X, ldx, beta, Y, ldy);
}

}  // namespace bkts

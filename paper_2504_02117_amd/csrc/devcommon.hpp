// Device-side helpers shared by the gfx950 kernels: XCD-aware block->tile mapping, the
// row-tile layout used by every block-vector kernel, and deterministic block reductions.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace bkts {
namespace dev {

constexpr int kThreads = 256;  // every tile kernel runs 4 wave64s per workgroup
constexpr int kXcd = 8;        // MI355X: 8 XCDs, workgroups dispatched round-robin over them

// Workgroups are dispatched round-robin over the XCDs; remap the dispatch index so that each XCD
// receives one contiguous range of slots (and its private L2 sees neighbouring rows).
__device__ __forceinline__ int64_t xcd_slot(int64_t b, int64_t nb) {
  const int64_t q = nb / kXcd, rem = nb % kXcd;
  const int64_t x = b % kXcd, i = b / kXcd;
  return x * q + (x < rem ? x : rem) + i;
}

// The 256-row chunks a workgroup of a persistent grid walks: the chunks are split into kXcd
// contiguous slabs, one per XCD (workgroup b runs on XCD b % kXcd), and the workgroups of an XCD
// step through its slab together (chunk j, j + W, j + 2W, ... for W workgroups per XCD), so each XCD
// works on one contiguous window at a time and the neighbour planes of its rows stay in its L2.
// Grids that are not a multiple of kXcd take one contiguous range per workgroup instead.
struct ChunkWalk {
  int64_t first, end, step;
};
__device__ __forceinline__ ChunkWalk xcd_chunks(int64_t chunks) {
  ChunkWalk w;
  if (gridDim.x % kXcd == 0) {
    const int64_t nw = gridDim.x / kXcd, x = blockIdx.x % kXcd, j = blockIdx.x / kXcd;
    const int64_t per = (chunks + kXcd - 1) / kXcd;
    const int64_t hi = (x + 1) * per < chunks ? (x + 1) * per : chunks;
    w.first = x * per + j;
    w.end = hi;
    w.step = nw;
  } else {
    const int64_t slot = xcd_slot(blockIdx.x, gridDim.x);
    const int64_t per = (chunks + gridDim.x - 1) / gridDim.x;
    w.first = slot * per;
    w.end = (slot + 1) * per < chunks ? (slot + 1) * per : chunks;
    w.step = 1;
  }
  return w;
}

// Row tiles of a block vector with padded width KP (power of two, 1..32).  A tile holds
// RT = 2048/KP rows.  Thread t owns column c = t % KP of rows t/KP + i*RS (RS = 256/KP),
// i = 0..7, both for its global loads and for its outputs, so loads are coalesced and each
// thread keeps its own elements in registers; only cross-column reads go through LDS.
template <int KP>
struct TileGeom {
  static_assert(KP == 1 || KP == 2 || KP == 4 || KP == 8 || KP == 16 || KP == 32, "KP");
  static constexpr int RT = 2048 / KP;          // rows per tile
  static constexpr int RS = kThreads / KP;      // row stride between a thread's rows
  static constexpr int RPT = RT / RS;           // rows per thread (= 8)
  static constexpr int LDL = (KP >= 2) ? KP + 2 : 1;  // LDS row stride in doubles (16-byte aligned rows)
  static constexpr int LDS_DOUBLES = RT * LDL;
};

template <typename T>
__device__ __forceinline__ double ld_d(const T* p) { return static_cast<double>(*p); }

// Dot product of LDS tile row `row` (k valid columns, zero padded to KP) with a register column.
template <int KP>
__device__ __forceinline__ double lds_row_dot(const double* lds, int row, const double (&col)[KP]) {
  using G = TileGeom<KP>;
  const double* p = lds + row * G::LDL;
  double s = 0.0;
  if constexpr (KP == 1) {
    s = p[0] * col[0];
  } else {
#pragma unroll
    for (int j = 0; j < KP; j += 2) {
      const double2 v = *reinterpret_cast<const double2*>(p + j);
      s = fma(v.x, col[j], s);
      s = fma(v.y, col[j + 1], s);
    }
  }
  return s;
}

// acc[a] += lds_row[a] * y  for a < KP  (Gram accumulation of column c owned by the thread)
template <int KP>
__device__ __forceinline__ void lds_row_axpy(const double* lds, int row, double y, double (&acc)[KP]) {
  using G = TileGeom<KP>;
  const double* p = lds + row * G::LDL;
  if constexpr (KP == 1) {
    acc[0] = fma(p[0], y, acc[0]);
  } else {
#pragma unroll
    for (int j = 0; j < KP; j += 2) {
      const double2 v = *reinterpret_cast<const double2*>(p + j);
      acc[j] = fma(v.x, y, acc[j]);
      acc[j + 1] = fma(v.y, y, acc[j + 1]);
    }
  }
}

// Reduce per-thread accumulators acc[0..NA) (thread column c = t % KP) over all threads of the
// block that share c, in a fixed order, and store entry (a, c) to partials[(a*KP + c)*nslots + slot].
// `red` must hold 4*NA*KP doubles of LDS.  Ends with a barrier.
template <int KP, int NA>
__device__ __forceinline__ void block_reduce_store(double (&acc)[NA], double* red, double* partials,
                                                   int64_t nslots, int64_t slot) {
  const int t = threadIdx.x;
#pragma unroll
  for (int off = KP; off < 64; off <<= 1) {
#pragma unroll
    for (int a = 0; a < NA; ++a) acc[a] += __shfl_xor(acc[a], off);
  }
  const int w = t >> 6, lane = t & 63;
  if (lane < KP) {
#pragma unroll
    for (int a = 0; a < NA; ++a) red[(w * NA + a) * KP + lane] = acc[a];
  }
  __syncthreads();
  for (int e = t; e < NA * KP; e += kThreads) {
    const double s = ((red[e] + red[NA * KP + e]) + red[2 * NA * KP + e]) + red[3 * NA * KP + e];
    partials[(int64_t)e * nslots + slot] = s;
  }
  __syncthreads();
}

}  // namespace dev
}  // namespace bkts

// Blocked SpMV core for gfx950 (paper §4.2: one index per dense block).
//
// A group of G lanes (G a power of two dividing the 64-lane wavefront) owns one
// block row.  Lane l takes blocks k0+l, k0+l+G, ... of the row: consecutive lanes
// read consecutive blocks, so a wave's value loads cover one contiguous stretch of
// the value array.  Each lane keeps one whole block in registers, gathers the
// BC*NRHS entries of x it multiplies, and accumulates BR*NRHS partial sums; the
// group then reduces them with cross-lane shuffles (no LDS, no atomics), so the
// result is deterministic.  The per-row epilogue is a template parameter, which
// lets the smoother, residual and CG kernels fuse their vector updates into the
// product instead of making extra passes over HBM.
#pragma once

#include <algorithm>

#include "internal.hpp"

namespace blk {

constexpr int kBlock = 256;

template <class T>
__device__ __forceinline__ T fmadd(T a, T b, T c) { return a * b + c; }

template <int N, class T>
__device__ __forceinline__ T pick(const T (&v)[N], int i) {
  T r = T(0);
#pragma unroll
  for (int t = 0; t < N; ++t)
    if (t == i) r = v[t];
  return r;
}

template <int BR, int BC, int NR, class TM, class TX, class TA>
__device__ __forceinline__ void block_fma(const TM* __restrict__ b, const TA (&xv)[BC * NR], TA (&acc)[BR * NR]) {
#pragma unroll
  for (int i = 0; i < BR; ++i) {
#pragma unroll
    for (int j = 0; j < BC; ++j) {
      const TA a = ld<TA>(b + i * BC + j);
#pragma unroll
      for (int q = 0; q < NR; ++q) acc[i * NR + q] = fmadd(a, xv[j * NR + q], acc[i * NR + q]);
    }
  }
}

// Lanes of a group stride over the blocks of the row; each lane takes U blocks per
// step and issues all their loads before the multiply-adds, so a wave keeps
// U * 64 blocks of loads in flight.
//
// SYM (square blocks, a structurally symmetric matrix): the strictly lower blocks
// of the row are not read from their own position but as the transpose of their
// mirror in the upper triangle, mir[k] = position of block (colidx[k], row).  Only
// the upper triangle and the diagonal are then streamed from HBM; each mirrored
// block was read by its own (earlier) row shortly before, so its second read is
// mostly served by the caches.  For a symmetric matrix the products are the same,
// in the same order within a lane.
template <int BR, int BC, int NR, int G, int U, class TM, class TX, class TA, bool SYM = false>
__device__ __forceinline__ void row_product(const int32_t* __restrict__ colidx,
                                            const TM* __restrict__ val, const TX* __restrict__ x,
                                            int k0, int k1, int lane, TA (&acc)[BR * NR], int row = 0,
                                            const int32_t* __restrict__ mir = nullptr) {
  static_assert(!SYM || BR == BC, "symmetric reads need square blocks");
#pragma unroll
  for (int t = 0; t < BR * NR; ++t) acc[t] = TA(0);
  for (int kb = k0 + lane; kb < k1; kb += G * U) {
    TM bv[U][BR * BC];
    TA xv[U][BC * NR];
    bool low[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int k = kb + u * G;
      low[u] = false;
      if (k < k1) {
        // with symmetric reads the block's source position comes from the mirror index
        // (k itself for the diagonal and upper blocks), loaded alongside the column
        // index, so the value load waits for one index load as in the full reads
        const int c = colidx[k];
        int src = k;
        if constexpr (SYM) src = mir[k];
        const TX* xc = x + static_cast<size_t>(c) * (BC * NR);
#pragma unroll
        for (int t = 0; t < BC * NR; ++t) xv[u][t] = ld<TA>(xc + t);
        if constexpr (SYM) low[u] = c < row;
        const TM* b = val + static_cast<size_t>(src) * (BR * BC);
#pragma unroll
        for (int t = 0; t < BR * BC; ++t) bv[u][t] = b[t];
      } else {
#pragma unroll
        for (int t = 0; t < BC * NR; ++t) xv[u][t] = TA(0);
#pragma unroll
        for (int t = 0; t < BR * BC; ++t) bv[u][t] = TM{};
      }
    }
    if constexpr (SYM) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
#pragma unroll
        for (int i = 0; i < BR; ++i) {
#pragma unroll
          for (int j = i + 1; j < BC; ++j) {
            const TM a = bv[u][i * BC + j], b = bv[u][j * BC + i];
            bv[u][i * BC + j] = low[u] ? b : a;
            bv[u][j * BC + i] = low[u] ? a : b;
          }
        }
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) block_fma<BR, BC, NR, TM, TX, TA>(bv[u], xv[u], acc);
  }
#pragma unroll
  for (int t = 0; t < BR * NR; ++t) acc[t] = group_sum<G>(acc[t]);
}

// Generic kernel: one tile of kBlock / G block rows per workgroup; logical
// workgroups are XCD-contiguous (the hardware hands workgroup b to XCD b mod 8 and
// each XCD has its own L2), so neighbouring rows, which gather the same x entries,
// run on the same XCD at the same time.  A reducing epilogue (dot products) leaves
// one partial sum per workgroup; every thread reaches that block reduction.
template <int BR, int BC, int NR, int G, int U, class TM, class TX, class TA, class Epi, bool SYM = false>
__global__ __launch_bounds__(kBlock) void spmv_kernel(int nbr, const int32_t* __restrict__ rowptr,
                                                      const int32_t* __restrict__ colidx,
                                                      const TM* __restrict__ val,
                                                      const TX* __restrict__ x, Epi epi,
                                                      const int32_t* __restrict__ mir = nullptr,
                                                      int chunk = kSpmvChunk) {
  constexpr int kRows = kBlock / G;
  const int lb = xcd_chunked_block(static_cast<int>(blockIdx.x), static_cast<int>(gridDim.x), chunk);
  const int row = lb * kRows + static_cast<int>(threadIdx.x) / G;
  const int lane = static_cast<int>(threadIdx.x) % G;
  TA acc[BR * NR];
  const bool active = row < nbr;
  // the row's extent is loaded first and the epilogue's own-row operands right after
  // it, before the product: loads complete in issue order, so waiting for the extent
  // does not wait for the operands, whose latency then overlaps the block loads
  int k0 = 0, k1 = 0;
  if (active) {
    k0 = rowptr[row];
    k1 = rowptr[row + 1];
  }
  const auto pre = epi.template prefetch<BR, NR, G>(active, row);
  if (active) {
    row_product<BR, BC, NR, G, U, TM, TX, TA, SYM>(colidx, val, x, k0, k1, lane, acc, row, mir);
  } else {
#pragma unroll
    for (int z = 0; z < BR * NR; ++z) acc[z] = TA(0);
  }
  const double part = epi.template apply<BR, NR, G>(active, row, lane, acc, pre);
  if constexpr (Epi::kReduce) {
    __shared__ double lds[4];
    const double sum = block_sum_256(part, lds);
    if (threadIdx.x == 0) epi.partial[lb] = sum;
  }
}


// Eight right-hand sides, G lanes per block row, one block per lane and step (as
// with one right-hand side, so a wave's block loads cover one contiguous stretch).
// Each lane multiplies its block with the whole 8-column panel of x (contiguous) into
// BR x 8 partial sums kept column by column, v[q * BR + i].  The G lanes are then
// added by an xor tree down to 8 lanes, and the last three levels are a
// reduce-scatter: at offset 4, 2, 1 a lane keeps the half of the columns selected by
// its own lane bit and adds the other lane's copy of that half, so lane q ends with
// the BR sums of column q (BR * 8 * 7 / 8 shuffles instead of BR * 8 * 3).  Lanes
// 0..7 then own the row's outputs, column by column, so the epilogue's block-row
// arithmetic (D^-1 r) stays inside a lane.
template <int BR, int BC, int G, int U, class TM, class TX, class TA, class Epi>
__global__ __launch_bounds__(kBlock) void spmm8_kernel(int nbr, const int32_t* __restrict__ rowptr,
                                                       const int32_t* __restrict__ colidx,
                                                       const TM* __restrict__ val,
                                                       const TX* __restrict__ x, Epi epi) {
  constexpr int NR = 8;
  static_assert(G >= NR, "eight right-hand sides need G >= 8");
  constexpr int kRows = kBlock / G;
  const int lb = xcd_chunked_block(static_cast<int>(blockIdx.x), static_cast<int>(gridDim.x), kSpmvChunk);
  const int row = lb * kRows + static_cast<int>(threadIdx.x) / G;
  const int lane = static_cast<int>(threadIdx.x) % G;
  TA v[NR * BR];  // v[q * BR + i]: row i of the block row, column q
#pragma unroll
  for (int t = 0; t < NR * BR; ++t) v[t] = TA(0);
  const bool active = row < nbr;
  if (active) {
    const int k1 = rowptr[row + 1];
    for (int kb = rowptr[row] + lane; kb < k1; kb += G * U) {
      TM bv[U][BR * BC];
      TA xv[U][BC * NR];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int k = kb + u * G;
        if (k < k1) {
          const TX* xc = x + static_cast<size_t>(colidx[k]) * (BC * NR);
#pragma unroll
          for (int t = 0; t < BC * NR; ++t) xv[u][t] = ld<TA>(xc + t);
          const TM* b = val + static_cast<size_t>(k) * (BR * BC);
#pragma unroll
          for (int t = 0; t < BR * BC; ++t) bv[u][t] = b[t];
        } else {
#pragma unroll
          for (int t = 0; t < BC * NR; ++t) xv[u][t] = TA(0);
#pragma unroll
          for (int t = 0; t < BR * BC; ++t) bv[u][t] = TM{};
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
#pragma unroll
        for (int i = 0; i < BR; ++i) {
#pragma unroll
          for (int j = 0; j < BC; ++j) {
            const TA a = ld<TA>(&bv[u][i * BC + j]);
#pragma unroll
            for (int q = 0; q < NR; ++q) v[q * BR + i] = fmadd(a, xv[u][j * NR + q], v[q * BR + i]);
          }
        }
      }
    }
  }
  // full sums down to 8 lanes
#pragma unroll
  for (int off = G / 2; off >= NR; off >>= 1) {
#pragma unroll
    for (int t = 0; t < NR * BR; ++t) v[t] += __shfl_xor(v[t], off, G);
  }
  // reduce-scatter over the columns: offsets 4, 2, 1 halve the columns a lane keeps
  constexpr int H4 = 4 * BR, H2 = 2 * BR, H1 = BR;
  const bool b4 = (lane & 4) != 0, b2 = (lane & 2) != 0, b1 = (lane & 1) != 0;
  TA w4[H4];
#pragma unroll
  for (int t = 0; t < H4; ++t) {
    const TA send = b4 ? v[t] : v[H4 + t];
    const TA keep = b4 ? v[H4 + t] : v[t];
    w4[t] = keep + __shfl_xor(send, 4, G);
  }
  TA w2[H2];
#pragma unroll
  for (int t = 0; t < H2; ++t) {
    const TA send = b2 ? w4[t] : w4[H2 + t];
    const TA keep = b2 ? w4[H2 + t] : w4[t];
    w2[t] = keep + __shfl_xor(send, 2, G);
  }
  TA acc[BR];
#pragma unroll
  for (int t = 0; t < H1; ++t) {
    const TA send = b1 ? w2[t] : w2[H1 + t];
    const TA keep = b1 ? w2[H1 + t] : w2[t];
    acc[t] = keep + __shfl_xor(send, 1, G);
  }
  epi.template apply8<BR, G>(active, row, lane, acc);
}

// mir != nullptr selects the symmetric reads (one right-hand side, square blocks;
// ignored otherwise).  Their workgroup runs per XCD then span sym_dist / 8 rows (one
// eighth of the matrix's typical lower bandwidth, e.g. one node plane of a 3D mesh in
// natural order): run r + 8, the next run of the same XCD, holds the rows sym_dist
// further on, whose mirrored lower blocks run r has just streamed into that XCD's L2.
template <int BR, int BC, int NR, int G, int U, class TM, class TX, class TA, class Epi>
int launch_g(int nbr, const int32_t* rowptr, const int32_t* colidx, const TM* val, const TX* x, const Epi& epi,
             hipStream_t s, const int32_t* mir, int sym_dist) {
  const int grid = ceil_div(nbr, kBlock / G);
  constexpr int kRows = kBlock / G;
  const int sym_chunk =
      sym_dist > 0 ? std::max(1, std::min(1 << 16, (sym_dist + kNumXcd * kRows / 2) / (kNumXcd * kRows))) : kSpmvChunk;
  if constexpr (NR == 8) {
    static_assert(!Epi::kReduce, "reducing epilogues take one right-hand side");
    spmm8_kernel<BR, BC, G, U, TM, TX, TA, Epi><<<grid, kBlock, 0, s>>>(nbr, rowptr, colidx, val, x, epi);
  } else if constexpr (BR == BC) {
    if (mir)
      spmv_kernel<BR, BC, NR, G, U, TM, TX, TA, Epi, true><<<grid, kBlock, 0, s>>>(nbr, rowptr, colidx, val, x, epi,
                                                                                    mir, sym_chunk);
    else
      spmv_kernel<BR, BC, NR, G, U, TM, TX, TA, Epi><<<grid, kBlock, 0, s>>>(nbr, rowptr, colidx, val, x, epi);
  } else {
    spmv_kernel<BR, BC, NR, G, U, TM, TX, TA, Epi><<<grid, kBlock, 0, s>>>(nbr, rowptr, colidx, val, x, epi);
  }
  return grid;
}

// Lane configuration: G lanes per block row (power of two, <= 64), U blocks per lane
// per step.  Encoded as G * 8 + U.
inline int lane_code(int G, int U) { return G * 8 + U; }

// Every lane code launch_rows compiles.
constexpr int kLaneCodes[] = {8 * 8 + 1, 8 * 8 + 2, 16 * 8 + 1, 16 * 8 + 2, 32 * 8 + 1, 32 * 8 + 2, 64 * 8 + 1, 64 * 8 + 2};

// Launch spmv_kernel with (G, U) chosen at run time; returns the number of
// workgroups (= number of partial sums written by a reducing epilogue).
template <int BR, int BC, int NR, class TM, class TX, class TA, class Epi>
int launch_rows(int code, int nbr, const int32_t* rowptr, const int32_t* colidx, const TM* val, const TX* x,
                const Epi& epi, hipStream_t s, const int32_t* mir = nullptr, int sym_dist = 0) {
  if (nbr <= 0) return 0;
  int grid;
  switch (code) {
#define BLK_CASE(GG, UU)                                                                                        \
  case GG * 8 + UU:                                                                                             \
    grid = launch_g<BR, BC, NR, GG, UU, TM, TX, TA, Epi>(nbr, rowptr, colidx, val, x, epi, s, mir, sym_dist);   \
    break;
    BLK_CASE(8, 1)
    BLK_CASE(8, 2)
    BLK_CASE(16, 1)
    BLK_CASE(16, 2)
    BLK_CASE(32, 1)
    BLK_CASE(32, 2)
    BLK_CASE(64, 1)
    BLK_CASE(64, 2)
#undef BLK_CASE
    default:
      grid = launch_g<BR, BC, NR, 64, 2, TM, TX, TA, Epi>(nbr, rowptr, colidx, val, x, epi, s, mir, sym_dist);
      break;
  }
  HIP_CHECK(hipGetLastError());
  return grid;
}

inline int grid_for(int G, int nbr) { return ceil_div(nbr, kBlock / G); }

// Epilogues implement
//   prefetch<BR,NR,G>(active, row) -> Pre   (own-row operands, loaded early)
//   apply<BR,NR,G>(active, row, lane, acc, pre) -> contribution to a block sum
// and set kReduce when the contributions are to be summed (partial[] per block).
struct NoPre {};

template <class T, int N>
struct RowVals {
  T v[N];
};

// When the BR * NR outputs of a row fit in its lane group (BR * NR <= G), lane l < BR * NR
// owns output l: it alone loads that output's own-row operands and stores it, instead
// of every lane of the group loading all of them.
template <int N, int G>
constexpr bool lane_owned() { return N <= G; }

// y = alpha * (A x) + beta * y
template <class TY, class TA>
struct EpiAxpby {
  static constexpr bool kReduce = false;
  TY* __restrict__ y;
  TA alpha, beta;
  double* partial = nullptr;
  template <int BR, int NR, int G>
  static constexpr int pre_len() { return lane_owned<BR * NR, G>() ? 1 : BR * NR; }
  template <int BR, int NR, int G>
  __device__ __forceinline__ RowVals<TA, pre_len<BR, NR, G>()> prefetch(bool active, int row) const {
    constexpr int N = BR * NR;
    RowVals<TA, pre_len<BR, NR, G>()> p;
#pragma unroll
    for (int t = 0; t < pre_len<BR, NR, G>(); ++t) p.v[t] = TA(0);
    if (!active || beta == TA(0)) return p;
    if constexpr (lane_owned<N, G>()) {
      const int lane = min(static_cast<int>(threadIdx.x) % G, N - 1);
      p.v[0] = ld<TA>(y + static_cast<size_t>(row) * N + lane);
    } else {
#pragma unroll
      for (int t = 0; t < N; ++t) p.v[t] = ld<TA>(y + static_cast<size_t>(row) * N + t);
    }
    return p;
  }
  template <int BR, int NR, int G>
  __device__ __forceinline__ double apply(bool active, int row, int lane, const TA (&acc)[BR * NR],
                                          const RowVals<TA, pre_len<BR, NR, G>()>& pre) const {
    constexpr int N = BR * NR;
    if (!active) return 0.0;
    if constexpr (lane_owned<N, G>()) {
      if (lane < N) {
        TA v = alpha * pick<N>(acc, lane);
        if (beta != TA(0)) v = fmadd(beta, pre.v[0], v);
        st(y + static_cast<size_t>(row) * N + lane, v);
      }
    } else {
#pragma unroll
      for (int l = 0; l < N; ++l) {
        if ((l % G) != lane) continue;
        TA v = alpha * acc[l];
        if (beta != TA(0)) v = fmadd(beta, pre.v[l], v);
        st(y + static_cast<size_t>(row) * N + l, v);
      }
    }
    return 0.0;
  }
  // eight right-hand sides, column-lane layout: lane q < 8 owns column q of the row
  template <int BR, int G>
  __device__ __forceinline__ void apply8(bool active, int row, int lane, const TA (&acc)[BR]) const {
    if (!active || lane >= 8) return;
    const size_t base = static_cast<size_t>(row) * (BR * 8) + lane;
#pragma unroll
    for (int i = 0; i < BR; ++i) {
      TA v = alpha * acc[i];
      if (beta != TA(0)) v = fmadd(beta, ld<TA>(y + base + i * 8), v);
      st(y + base + i * 8, v);
    }
  }
};

}  // namespace blk

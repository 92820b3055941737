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
template <int BR, int BC, int NR, int G, int U, class TM, class TX, class TA>
__device__ __forceinline__ void row_product(const int32_t* __restrict__ rowptr,
                                            const int32_t* __restrict__ colidx,
                                            const TM* __restrict__ val, const TX* __restrict__ x,
                                            int row, int lane, TA (&acc)[BR * NR]) {
#pragma unroll
  for (int t = 0; t < BR * NR; ++t) acc[t] = TA(0);
  const int k0 = rowptr[row], k1 = rowptr[row + 1];
  for (int kb = k0 + lane; kb < k1; kb += G * U) {
    TM bv[U][BR * BC];
    TA xv[U][BC * NR];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int k = kb + u * G;
      if (k < k1) {
        const int c = colidx[k];
        const TX* xc = x + static_cast<size_t>(c) * (BC * NR);
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
template <int BR, int BC, int NR, int G, int U, class TM, class TX, class TA, class Epi>
__global__ __launch_bounds__(kBlock) void spmv_kernel(int nbr, const int32_t* __restrict__ rowptr,
                                                      const int32_t* __restrict__ colidx,
                                                      const TM* __restrict__ val,
                                                      const TX* __restrict__ x, Epi epi) {
  constexpr int kRows = kBlock / G;
  const int lb = xcd_logical_block(blockIdx.x, gridDim.x);
  const int row = lb * kRows + static_cast<int>(threadIdx.x) / G;
  const int lane = static_cast<int>(threadIdx.x) % G;
  TA acc[BR * NR];
  const bool active = row < nbr;
  // the epilogue's own-row operands are loaded before the product so that their
  // latency overlaps the block loads instead of following the row reduction
  const auto pre = epi.template prefetch<BR, NR, G>(active, row);
  if (active) {
    row_product<BR, BC, NR, G, U, TM, TX, TA>(rowptr, colidx, val, x, row, lane, acc);
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


template <int BR, int BC, int NR, int G, int U, class TM, class TX, class TA, class Epi>
int launch_g(int nbr, const int32_t* rowptr, const int32_t* colidx, const TM* val, const TX* x, const Epi& epi,
             hipStream_t s) {
  const int grid = ceil_div(nbr, kBlock / G);
  spmv_kernel<BR, BC, NR, G, U, TM, TX, TA, Epi><<<grid, kBlock, 0, s>>>(nbr, rowptr, colidx, val, x, epi);
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
                const Epi& epi, hipStream_t s) {
  if (nbr <= 0) return 0;
  int grid;
  switch (code) {
#define BLK_CASE(GG, UU)                                                                                        \
  case GG * 8 + UU:                                                                                             \
    grid = launch_g<BR, BC, NR, GG, UU, TM, TX, TA, Epi>(nbr, rowptr, colidx, val, x, epi, s);                  \
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
      grid = launch_g<BR, BC, NR, 64, 2, TM, TX, TA, Epi>(nbr, rowptr, colidx, val, x, epi, s);
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

// y = alpha * (A x) + beta * y
template <class TY, class TA>
struct EpiAxpby {
  static constexpr bool kReduce = false;
  TY* __restrict__ y;
  TA alpha, beta;
  double* partial = nullptr;
  template <int BR, int NR, int G>
  __device__ __forceinline__ RowVals<TA, BR * NR> prefetch(bool active, int row) const {
    RowVals<TA, BR * NR> p;
#pragma unroll
    for (int t = 0; t < BR * NR; ++t) p.v[t] = TA(0);
    if (active && beta != TA(0)) {
#pragma unroll
      for (int t = 0; t < BR * NR; ++t) p.v[t] = ld<TA>(y + static_cast<size_t>(row) * (BR * NR) + t);
    }
    return p;
  }
  template <int BR, int NR, int G>
  __device__ __forceinline__ double apply(bool active, int row, int lane, const TA (&acc)[BR * NR],
                                          const RowVals<TA, BR * NR>& pre) const {
    if (!active) return 0.0;
#pragma unroll
    for (int l = 0; l < BR * NR; ++l) {
      if ((l % G) != lane) continue;
      const size_t o = static_cast<size_t>(row) * (BR * NR) + l;
      TA v = alpha * acc[l];
      if (beta != TA(0)) v = fmadd(beta, pre.v[l], v);
      st(y + o, v);
    }
    return 0.0;
  }
};

}  // namespace blk

// Galerkin coarse operator A_c = P^T A P on a fixed block pattern (paper §2.1,
// §3.1, §3.5).  The symbolic phase (host) builds the pattern of A P and of A_c and
// keeps it; the numeric phase is device-only, allocation-free and deterministic:
//   pass 1: AP_ib = sum_j A_ij P_jb          (one lane per output block of AP)
//   pass 2: C_ac  = sum_i R_ai AP_ic, R = P^T (one lane per output block of C)
// The transpose R comes from P's value-stamped cache, so a recompute with an
// unchanged prolongator never rebuilds prolongator-side data (paper §3.5).
#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <thread>
#include <string>
#include <type_traits>

#include "ptap_plan.hpp"
#include "spmv_core.hpp"

namespace blk {

namespace {

__device__ __forceinline__ int search(const int32_t* __restrict__ cols, int lo, int hi, int key) {
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    const int v = cols[mid];
    if (v == key) return mid;
    if (v < key) lo = mid + 1; else hi = mid;
  }
  return -1;
}

// pass 1: AP = A P.  Group of G lanes per row of AP, lane per output block.
template <int BR, int BC, int G, class TA_, class TP, class TA>
__global__ __launch_bounds__(kBlock) void ap_kernel(int nrows, const int32_t* __restrict__ a_rp,
                                                    const int32_t* __restrict__ a_ci, const TA_* __restrict__ a_v,
                                                    const int32_t* __restrict__ p_rp, const int32_t* __restrict__ p_ci,
                                                    const TP* __restrict__ p_v, const int32_t* __restrict__ ap_rp,
                                                    const int32_t* __restrict__ ap_ci, TA* __restrict__ ap_v) {
  const int lb = xcd_logical_block(blockIdx.x, gridDim.x);
  const int row = lb * (kBlock / G) + static_cast<int>(threadIdx.x) / G;
  const int lane = static_cast<int>(threadIdx.x) % G;
  if (row >= nrows) return;
  const int s0 = ap_rp[row], s1 = ap_rp[row + 1];
  const int k0 = a_rp[row], k1 = a_rp[row + 1];
  for (int sb = s0; sb < s1; sb += G) {
    const int s = sb + lane;
    if (s >= s1) break;
    const int b = ap_ci[s];
    TA acc[BR * BC];
#pragma unroll
    for (int t = 0; t < BR * BC; ++t) acc[t] = TA(0);
    for (int k = k0; k < k1; ++k) {
      const int j = a_ci[k];
      const int q = search(p_ci, p_rp[j], p_rp[j + 1], b);
      if (q < 0) continue;
      const TA_* ab = a_v + static_cast<size_t>(k) * (BR * BR);
      const TP* pb = p_v + static_cast<size_t>(q) * (BR * BC);
      TA pv[BR * BC];
#pragma unroll
      for (int t = 0; t < BR * BC; ++t) pv[t] = ld<TA>(pb + t);
#pragma unroll
      for (int r = 0; r < BR; ++r) {
#pragma unroll
        for (int m = 0; m < BR; ++m) {
          const TA a = ld<TA>(ab + r * BR + m);
#pragma unroll
          for (int c = 0; c < BC; ++c) acc[r * BC + c] = fmadd(a, pv[m * BC + c], acc[r * BC + c]);
        }
      }
    }
    TA* o = ap_v + static_cast<size_t>(s) * (BR * BC);
#pragma unroll
    for (int t = 0; t < BR * BC; ++t) o[t] = acc[t];
  }
}

// pass 2: C = R AP.  Group of G lanes per coarse row, lane per output block.
template <int BR, int BC, int G, class TR, class TA, class TC>
__global__ __launch_bounds__(kBlock) void rap_kernel(int ncoarse, const int32_t* __restrict__ r_rp,
                                                     const int32_t* __restrict__ r_ci, const TR* __restrict__ r_v,
                                                     const int32_t* __restrict__ ap_rp, const int32_t* __restrict__ ap_ci,
                                                     const TA* __restrict__ ap_v, const int32_t* __restrict__ c_rp,
                                                     const int32_t* __restrict__ c_ci, TC* __restrict__ c_v) {
  const int lb = xcd_logical_block(blockIdx.x, gridDim.x);
  const int row = lb * (kBlock / G) + static_cast<int>(threadIdx.x) / G;
  const int lane = static_cast<int>(threadIdx.x) % G;
  if (row >= ncoarse) return;
  const int s0 = c_rp[row], s1 = c_rp[row + 1];
  const int k0 = r_rp[row], k1 = r_rp[row + 1];
  for (int sb = s0; sb < s1; sb += G) {
    const int s = sb + lane;
    if (s >= s1) break;
    const int c = c_ci[s];
    TA acc[BC * BC];
#pragma unroll
    for (int t = 0; t < BC * BC; ++t) acc[t] = TA(0);
    for (int k = k0; k < k1; ++k) {
      const int i = r_ci[k];
      const int q = search(ap_ci, ap_rp[i], ap_rp[i + 1], c);
      if (q < 0) continue;
      const TR* rb = r_v + static_cast<size_t>(k) * (BC * BR);  // BC x BR block of R
      const TA* apb = ap_v + static_cast<size_t>(q) * (BR * BC);
      TA apv[BR * BC];
#pragma unroll
      for (int t = 0; t < BR * BC; ++t) apv[t] = apb[t];
#pragma unroll
      for (int r = 0; r < BC; ++r) {
#pragma unroll
        for (int m = 0; m < BR; ++m) {
          const TA a = ld<TA>(rb + r * BR + m);
#pragma unroll
          for (int cc = 0; cc < BC; ++cc) acc[r * BC + cc] = fmadd(a, apv[m * BC + cc], acc[r * BC + cc]);
        }
      }
    }
    TC* o = c_v + static_cast<size_t>(s) * (BC * BC);
#pragma unroll
    for (int t = 0; t < BC * BC; ++t) st(o + t, acc[t]);
  }
}

// NL lanes per output block (1 or 3).  A workgroup takes kBlock / NL consecutive output
// blocks, which belong to rows row0..row1 (row1 = first row of the next workgroup), and
// walks them in the order given by `perm` (sorted by contribution count at symbolic
// time, so the lanes of a wave run loops of similar length).  For every entry k of
// those rows of the first operand X (A or R), LDS holds ystart[k] = the start of the Y
// row it multiplies (P row a_ci[k], or AP row r_ci[k]); in the A P pass the X blocks of
// the rows are staged in LDS too (one coalesced copy).  The LDS is sized at symbolic
// time from the workgroups' extents (`cap` entries), so small blocks (FP32) leave room
// for more resident workgroups.  Y blocks are read with 16-byte (FP64) or 8-byte (FP32)
// vector loads when VEC is set.
#ifndef BLK_AP_XSTAGE_F64
#define BLK_AP_XSTAGE_F64 1
#endif
template <bool kIsAP, class TX>
constexpr bool kStageX = kIsAP && (sizeof(TX) == 4 || BLK_AP_XSTAGE_F64);

inline size_t ptap_lds_bytes(int cap, int xbytes) {
  return ((static_cast<size_t>(cap) * 4 + 15) & ~static_cast<size_t>(15)) + static_cast<size_t>(cap) * xbytes;
}

template <class T, bool VEC, int N>
__device__ __forceinline__ void load_y(const T* __restrict__ p, T (&v)[N]) {
  if constexpr (VEC && sizeof(T) == 8 && N % 2 == 0) {
    const double2* q = reinterpret_cast<const double2*>(p);
#pragma unroll
    for (int t = 0; t < N / 2; ++t) {
      const double2 d = q[t];
      v[2 * t] = d.x;
      v[2 * t + 1] = d.y;
    }
  } else if constexpr (VEC && sizeof(T) == 4 && N % 2 == 0) {
    const float2* q = reinterpret_cast<const float2*>(p);
#pragma unroll
    for (int t = 0; t < N / 2; ++t) {
      const float2 d = q[t];
      v[2 * t] = d.x;
      v[2 * t + 1] = d.y;
    }
  } else {
#pragma unroll
    for (int t = 0; t < N; ++t) v[t] = p[t];
  }
}

// The CW values of columns c0..c0+CW-1 of each of the R rows of a row-major block with
// BC columns (all of it when CW == BC).
template <class T, bool VEC, int R, int BC, int CW>
__device__ __forceinline__ void load_ycols(const T* __restrict__ p, int c0, T (&v)[R * CW]) {
#pragma unroll
  for (int r = 0; r < R; ++r) {
    T row[CW];
    load_y<T, VEC>(p + r * BC + c0, row);
#pragma unroll
    for (int c = 0; c < CW; ++c) v[r * CW + c] = row[c];
  }
}

template <int BR, int BC, class TX, class TY, class TA, class CT, bool kIsAP, bool VEC, int NL>
__global__ __launch_bounds__(kBlock) void pairs_slot_kernel(int64_t nslots, int nrows, const int32_t* __restrict__ slot_row0,
                                                            const uint8_t* __restrict__ perm,
                                                            const int32_t* __restrict__ x_rp,
                                                            const int32_t* __restrict__ x_ci, const TX* __restrict__ x_v,
                                                            const int32_t* __restrict__ y_rp, const TY* __restrict__ y_v,
                                                            const int32_t* __restrict__ o_rp,
                                                            const int32_t* __restrict__ pp, const CT* __restrict__ codes,
                                                            int shift, void* __restrict__ out,
                                                            const int32_t* __restrict__ out_idx,
                                                            const int32_t* __restrict__ mirror, int cap,
                                                            int xcd_chunk) {
  // kIsAP: X = A (BR x BR), Y = P (BR x BC), out AP (BR x BC) in TA
  // else : X = R (BC x BR), Y = AP (BR x BC), out C (BC x BC) in the type of A
  constexpr int XR = kIsAP ? BR : BC;  // rows of an X block
  constexpr int XC = BR;               // cols of an X block
  constexpr int XB = XR * XC;
  constexpr int OR = XR;               // rows of an output block
  // NL lanes per output block; lane m owns its columns m*CW .. m*CW+CW-1 and reads only
  // those columns of every contributing Y block, so one load instruction of a wave
  // covers whole Y rows of a few blocks (a few cache lines) instead of one 16-byte piece
  // of 64 different blocks.  Every lane of the block reads the whole X block.
  static_assert(BC % NL == 0, "lanes must split the columns evenly");
  constexpr int CW = BC / NL;
  constexpr int SPW = kBlock / NL;     // output blocks per workgroup
  // only the AP pass stages X (A rows: ~27 blocks per row); R rows are too long
  extern __shared__ __align__(16) unsigned char ptap_lds[];
  int32_t* ystart = reinterpret_cast<int32_t*>(ptap_lds);
  TX* xs = reinterpret_cast<TX*>(ptap_lds + ((cap * 4 + 15) & ~15));
  // xcd_map: each XCD takes a contiguous range of workgroups (its L2 sees neighbouring
  // rows); otherwise the hardware's round-robin order, where all XCDs work on one region
  // at a time and the shared MALL holds what they gather
  const int w = xcd_chunk < 0   ? xcd_logical_block(blockIdx.x, gridDim.x)
                : xcd_chunk == 0 ? static_cast<int>(blockIdx.x)
                                 : xcd_chunked_block(static_cast<int>(blockIdx.x), static_cast<int>(gridDim.x), xcd_chunk);
  const int64_t s_begin = static_cast<int64_t>(w) * SPW;
  const int row0 = slot_row0[w];
  const int row1 = min(nrows - 1, slot_row0[w + 1]);
  const int nr = row1 - row0 + 1;
  const int kbase = x_rp[row0];
  const int nk = x_rp[row1 + 1] - kbase;
  const bool staged = nr <= kMaxR && nk <= cap;
  const bool xstaged = kStageX<kIsAP, TX> && staged;
  // the output and X row pointers of the workgroup's rows, so a lane finds its row and
  // the row's X extent in LDS instead of by a chain of global loads
  __shared__ int32_t orp_s[kMaxR + 1], xrp_s[kMaxR + 1];
  const bool rows_staged = nr <= kMaxR;
  if (rows_staged && threadIdx.x <= static_cast<unsigned>(nr)) {
    orp_s[threadIdx.x] = o_rp[row0 + threadIdx.x];
    xrp_s[threadIdx.x] = x_rp[row0 + threadIdx.x];
  }
  // staging: each thread issues kSU independent loads before storing them, so a
  // workgroup's start costs a few memory latencies rather than one per element
  constexpr int kSU = 8;
  if (staged) {
    for (int t0 = threadIdx.x; t0 < nk; t0 += kBlock * kSU) {
      int c[kSU];
#pragma unroll
      for (int u = 0; u < kSU; ++u) c[u] = t0 + u * kBlock < nk ? x_ci[kbase + t0 + u * kBlock] : 0;
      int ys[kSU];
#pragma unroll
      for (int u = 0; u < kSU; ++u) ys[u] = t0 + u * kBlock < nk ? y_rp[c[u]] : 0;
#pragma unroll
      for (int u = 0; u < kSU; ++u)
        if (t0 + u * kBlock < nk) ystart[t0 + u * kBlock] = ys[u];
    }
  }
  if (xstaged) {
    const TX* src = x_v + static_cast<size_t>(kbase) * XB;
    const int total = nk * XB;
    for (int t0 = threadIdx.x; t0 < total; t0 += kBlock * kSU) {
      TX v[kSU];
#pragma unroll
      for (int u = 0; u < kSU; ++u) v[u] = t0 + u * kBlock < total ? src[t0 + u * kBlock] : TX{};
#pragma unroll
      for (int u = 0; u < kSU; ++u)
        if (t0 + u * kBlock < total) xs[t0 + u * kBlock] = v[u];
    }
  }
  __syncthreads();
  const int slot = static_cast<int>(threadIdx.x) / NL;
  const int lm = static_cast<int>(threadIdx.x) % NL;
  if (slot >= SPW || s_begin + slot >= nslots) return;
  const int64_t sidx = s_begin + perm[s_begin + slot];
  const int c0 = lm * CW;
  int row = row0;
  int k0;
  if (rows_staged) {
    int r = 0;
    while (orp_s[r + 1] <= sidx) ++r;
    row = row0 + r;
    k0 = xrp_s[r];
  } else {
    while (o_rp[row + 1] <= sidx) ++row;
    k0 = x_rp[row];
  }
  const uint32_t mask = (1u << shift) - 1u;
  TA acc[OR * CW];
#pragma unroll
  for (int t = 0; t < OR * CW; ++t) acc[t] = TA(0);
  const int e0 = pp[sidx], e1 = pp[sidx + 1];
  // PU contributions per step: their Y blocks (and X blocks read from global memory)
  // are all loaded before the multiply-adds, so each lane keeps PU gathers in flight;
  // depths measured at 128^3.  Large blocks keep one to stay within the VGPR file.
  constexpr int kYBytes = BR * BC * static_cast<int>(sizeof(TA));
#ifndef BLK_PU_SPLIT_AP
#define BLK_PU_SPLIT_AP 4
#endif
#ifndef BLK_PU_SPLIT_RAP
#define BLK_PU_SPLIT_RAP 2
#endif
#ifndef BLK_AP_PU_F64
#define BLK_AP_PU_F64 2
#endif
#ifndef BLK_RAP_PU_F64
#define BLK_RAP_PU_F64 2
#endif
#ifndef BLK_AP_PU_F32
#define BLK_AP_PU_F32 4
#endif
#ifndef BLK_RAP_PU_F32
#define BLK_RAP_PU_F32 4
#endif
  constexpr int PU_STAGED = NL > 1 ? (kIsAP ? BLK_PU_SPLIT_AP : BLK_PU_SPLIT_RAP)
                     : (kYBytes == 144 && kIsAP) ? BLK_AP_PU_F64
                     : (kYBytes == 144 && !kIsAP) ? BLK_RAP_PU_F64
                     : (kYBytes == 72 && kIsAP) ? BLK_AP_PU_F32
                     : (kYBytes == 72 && !kIsAP) ? BLK_RAP_PU_F32
                     : (kYBytes > 144 ? 1 : (kYBytes > 72 ? 2 : 4));
  auto contrib = [&](const TX* xb, const TY (&yraw)[BR * CW]) {
#pragma unroll
    for (int r = 0; r < OR; ++r) {
#pragma unroll
      for (int m = 0; m < XC; ++m) {
        const TA xv = ld<TA>(xb + r * XC + m);
#pragma unroll
        for (int cc = 0; cc < CW; ++cc) acc[r * CW + cc] = fmadd(xv, ld<TA>(&yraw[m * CW + cc]), acc[r * CW + cc]);
      }
    }
  };
  // The walk is instantiated separately for staged and unstaged workgroups, so the
  // reads of the staged tables compile to LDS instructions: through a pointer that may
  // address either memory they would become flat accesses, which occupy the same
  // vector-memory pipeline as the Y gathers.
  auto walk = [&](auto ys_staged, auto x_staged) {
    constexpr bool YS = decltype(ys_staged)::value;
    constexpr bool XS = decltype(x_staged)::value;
    // workgroups too large for the LDS tables are rare; one pair per step keeps their
    // instantiation from raising the kernel's register count
    constexpr int PU = YS ? PU_STAGED : 1;
    auto xblock = [&](int k) -> const TX* {
      if constexpr (XS) return xs + (k - kbase) * XB;
      else return x_v + static_cast<size_t>(k) * XB;
    };
    auto place = [&](uint32_t code, int& k, int& q) {
      k = k0 + static_cast<int>(code >> shift);
      int ys;
      if constexpr (YS) ys = ystart[k - kbase];
      else ys = y_rp[x_ci[k]];
      q = ys + static_cast<int>(code & mask);
    };
    int e = e0;
    if (e + PU <= e1) {
      uint32_t cn[PU];
#pragma unroll
      for (int u = 0; u < PU; ++u) cn[u] = codes[e + u];
      for (; e + PU <= e1; e += PU) {
        int k[PU], q[PU];
#pragma unroll
        for (int u = 0; u < PU; ++u) place(cn[u], k[u], q[u]);
        TY yraw[PU][BR * CW];
        TX xraw[XS ? 1 : PU][XB];  // X blocks from global memory are loaded with the Y blocks
#pragma unroll
        for (int u = 0; u < PU; ++u)
          load_ycols<TY, VEC, BR, BC, CW>(y_v + static_cast<size_t>(q[u]) * (BR * BC), c0, yraw[u]);
        if constexpr (!XS) {
#pragma unroll
          for (int u = 0; u < PU; ++u) {
            const TX* xb = xblock(k[u]);
#pragma unroll
            for (int t = 0; t < XB; ++t) xraw[u][t] = xb[t];
          }
        }
        // the next step's codes, clamped to this block's list (always a valid address)
#pragma unroll
        for (int u = 0; u < PU; ++u) cn[u] = codes[min(e + PU + u, e1 - 1)];
        // every load of the step is issued before the first multiply-add: without the
        // barrier the scheduler interleaves them to save registers, leaving only a
        // few gathers in flight per wave
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int u = 0; u < PU; ++u) contrib(XS ? xblock(k[u]) : xraw[XS ? 0 : u], yraw[u]);
      }
    }
    for (; e < e1; ++e) {
      int k, q;
      place(codes[e], k, q);
      TY yraw[BR * CW];
      load_ycols<TY, VEC, BR, BC, CW>(y_v + static_cast<size_t>(q) * (BR * BC), c0, yraw);
      contrib(xblock(k), yraw);
    }
  };
  if (staged) {
    if constexpr (kStageX<kIsAP, TX>) walk(std::true_type{}, std::true_type{});
    else walk(std::true_type{}, std::false_type{});
  } else {
    walk(std::false_type{}, std::false_type{});
  }
  if constexpr (kIsAP) {
    TA* o = static_cast<TA*>(out) + static_cast<size_t>(sidx) * (OR * BC) + c0;
#pragma unroll
    for (int r = 0; r < OR; ++r) {
#pragma unroll
      for (int cc = 0; cc < CW; ++cc) o[r * BC + cc] = acc[r * CW + cc];
    }
  } else {
    // symmetric mode: slot sidx is the out_idx[sidx]-th block of C; its transpose
    // also goes to block mirror[sidx] (-1 on the diagonal)
    using TC = typename std::conditional<sizeof(TA) == 8, double, float>::type;
    const int64_t oi = out_idx ? out_idx[sidx] : sidx;
    TC* o = static_cast<TC*>(out) + static_cast<size_t>(oi) * (OR * BC) + c0;
#pragma unroll
    for (int r = 0; r < OR; ++r) {
#pragma unroll
      for (int cc = 0; cc < CW; ++cc) st(o + r * BC + cc, acc[r * CW + cc]);
    }
    if (mirror) {
      const int mi = mirror[sidx];
      if (mi >= 0) {
        TC* o2 = static_cast<TC*>(out) + static_cast<size_t>(mi) * (OR * BC);
#pragma unroll
        for (int r = 0; r < OR; ++r) {
#pragma unroll
          for (int cc = 0; cc < CW; ++cc) st(o2 + (c0 + cc) * OR + r, acc[r * CW + cc]);
        }
      }
    }
  }
}

inline bool aligned(const void* p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

template <int BR, int BC, class TA_, class TP, class TA, class CT>
void launch_ap_pairs(const PtapPlan& pl, const bsr_s* A, const bsr_s* P, TA* ap, hipStream_t s) {
  const int64_t ns = pl.ap_nslots;
  const int spw = kBlock / pl.ap_nl;
  const int grid = static_cast<int>((ns + spw - 1) / spw);
  if (grid == 0) return;
  // P blocks (BR*BC values) can be read with 2-element vector loads when the block
  // size is even and the array is aligned for it
  const bool vec = pl.ap_vec && (BR * BC) % 2 == 0 && aligned(P->val, 2 * sizeof(TP)) && sizeof(TP) >= 4;
  const size_t lds = ptap_lds_bytes(pl.ap_cap, kStageX<true, TA_> ? BR * BR * static_cast<int>(sizeof(TA_)) : 0);
#define BLK_APK(V, NL)                                                                                               \
  pairs_slot_kernel<BR, BC, TA_, TP, TA, CT, true, V, NL><<<grid, kBlock, lds, s>>>(                                      \
      ns, A->nbr, pl.ap_slot_row0.p, pl.ap_perm.p, A->rowptr, A->colidx, static_cast<const TA_*>(A->val), P->rowptr, \
      static_cast<const TP*>(P->val), pl.ap_rowptr.p, pl.ap_pairs.ptr.p,                                             \
      reinterpret_cast<const CT*>(pl.ap_pairs.codes.p), pl.ap_pairs.shift, ap, nullptr, nullptr, pl.ap_cap,      \
      pl.ap_xcd)
  if (pl.ap_nl == 3) {
    if (vec) BLK_APK(true, 3); else BLK_APK(false, 3);
  } else {
    if (vec) BLK_APK(true, 1); else BLK_APK(false, 1);
  }
#undef BLK_APK
}

template <int BR, int BC, class TA_, class TP, class TA, class CT>
void launch_rap_pairs(const PtapPlan& pl, const bsr_s* R, const bsr_s* C, const TA* ap, hipStream_t s) {
  const int64_t ns = pl.sym ? pl.c_nslots : C->nnzb;
  const int spw = kBlock / pl.c_nl;
  const int grid = static_cast<int>((ns + spw - 1) / spw);
  if (grid == 0) return;
  const int32_t* orp = pl.sym ? pl.c_up_rp.p : C->rowptr;
  const size_t lds = ptap_lds_bytes(pl.c_cap, 0);
#define BLK_RAPK(V, NL)                                                                                              \
  pairs_slot_kernel<BR, BC, TP, TA, TA, CT, false, V, NL><<<grid, kBlock, lds, s>>>(                                      \
      ns, C->nbr, pl.c_slot_row0.p, pl.c_perm.p, R->rowptr, R->colidx, static_cast<const TP*>(R->val), pl.ap_rowptr.p, \
      ap, orp, pl.c_pairs.ptr.p, reinterpret_cast<const CT*>(pl.c_pairs.codes.p), pl.c_pairs.shift, C->val,           \
      pl.sym ? pl.c_up_idx.p : nullptr, pl.sym ? pl.c_mirror.p : nullptr, pl.c_cap, pl.c_xcd)
  if (pl.c_nl == 3) {
    if (pl.c_vec) BLK_RAPK(true, 3); else BLK_RAPK(false, 3);
  } else {
    if (pl.c_vec) BLK_RAPK(true, 1); else BLK_RAPK(false, 1);
  }
#undef BLK_RAPK
}

template <int BR, int BC, class TA_, class TP, class TA>
void run_numeric(const PtapPlan& pl, const bsr_s* A, const bsr_s* P, const bsr_s* R, bsr_s* C, hipStream_t s) {
  TA* ap = reinterpret_cast<TA*>(pl.ap_val.p);
  if (A->nbr > 0) {
    switch (pl.ap_pairs.width) {
      case 1: launch_ap_pairs<BR, BC, TA_, TP, TA, uint8_t>(pl, A, P, ap, s); break;
      case 2: launch_ap_pairs<BR, BC, TA_, TP, TA, uint16_t>(pl, A, P, ap, s); break;
      case 4: launch_ap_pairs<BR, BC, TA_, TP, TA, uint32_t>(pl, A, P, ap, s); break;
      default:
#define BLK_AP(GG)                                                                                      \
  ap_kernel<BR, BC, GG, TA_, TP, TA><<<grid_for(GG, A->nbr), kBlock, 0, s>>>(                            \
      A->nbr, A->rowptr, A->colidx, static_cast<const TA_*>(A->val), P->rowptr, P->colidx,               \
      static_cast<const TP*>(P->val), pl.ap_rowptr.p, pl.ap_colidx.p, ap)
        if (pl.g_ap == 16) BLK_AP(16); else BLK_AP(32);
#undef BLK_AP
    }
    HIP_CHECK(hipGetLastError());
  }
  if (C->nbr > 0) {
    switch (pl.c_pairs.width) {
      case 1: launch_rap_pairs<BR, BC, TA_, TP, TA, uint8_t>(pl, R, C, ap, s); break;
      case 2: launch_rap_pairs<BR, BC, TA_, TP, TA, uint16_t>(pl, R, C, ap, s); break;
      case 4: launch_rap_pairs<BR, BC, TA_, TP, TA, uint32_t>(pl, R, C, ap, s); break;
      default:
#define BLK_RAP(GG)                                                                                     \
  rap_kernel<BR, BC, GG, TP, TA, TA_><<<grid_for(GG, C->nbr), kBlock, 0, s>>>(                           \
      C->nbr, R->rowptr, R->colidx, static_cast<const TP*>(R->val), pl.ap_rowptr.p, pl.ap_colidx.p, ap,  \
      C->rowptr, C->colidx, static_cast<TA_*>(C->val))
        if (pl.g_c == 16) BLK_RAP(16); else BLK_RAP(32);
#undef BLK_RAP
    }
    HIP_CHECK(hipGetLastError());
  }
}

template <int BR, int BC>
void numeric_shape(const PtapPlan& pl, const bsr_s* A, const bsr_s* P, const bsr_s* R, bsr_s* C, hipStream_t s) {
  if (A->dtype == BLKAMG_F64)
    run_numeric<BR, BC, double, double, double>(pl, A, P, R, C, s);
  else if (P->dtype == BLKAMG_F32)
    run_numeric<BR, BC, float, float, float>(pl, A, P, R, C, s);
  else
    run_numeric<BR, BC, float, bf16, float>(pl, A, P, R, C, s);
}

int pick_lanes(double avg) { return avg <= 16.0 ? 16 : 32; }

}  // namespace

// Structural product of two host patterns (sorted rows, no dropping).
void structural_product_host(int32_t nra, const std::vector<int32_t>& rpa, const std::vector<int32_t>& cia,
                             int32_t ncb, const std::vector<int32_t>& rpb, const std::vector<int32_t>& cib,
                             std::vector<int32_t>& rpc, std::vector<int32_t>& cic) {
  rpc.assign(static_cast<size_t>(nra) + 1, 0);
  cic.clear();
  std::vector<int32_t> mark(static_cast<size_t>(ncb), -1);
  std::vector<int32_t> row;
  for (int32_t i = 0; i < nra; ++i) {
    row.clear();
    for (int32_t k = rpa[i]; k < rpa[i + 1]; ++k) {
      const int32_t j = cia[k];
      for (int32_t q = rpb[j]; q < rpb[j + 1]; ++q) {
        const int32_t c = cib[q];
        if (mark[c] != i) {
          mark[c] = i;
          row.push_back(c);
        }
      }
    }
    std::sort(row.begin(), row.end());
    cic.insert(cic.end(), row.begin(), row.end());
    BLK_REQUIRE(cic.size() <= static_cast<size_t>(INT32_MAX), BLKAMG_EINVAL, "product pattern too large");
    rpc[i + 1] = static_cast<int32_t>(cic.size());
  }
}

namespace {

template <class F>
void parallel_rows(int32_t n, F&& f) {
  const int nth = std::max(1, std::min<int>(16, static_cast<int>(std::thread::hardware_concurrency())));
  if (n < 4096 || nth == 1) {
    f(0, n, 0);
    return;
  }
  std::vector<std::thread> ts;
  for (int t = 0; t < nth; ++t)
    ts.emplace_back([&, t] { f(static_cast<int32_t>(static_cast<int64_t>(n) * t / nth),
                               static_cast<int32_t>(static_cast<int64_t>(n) * (t + 1) / nth), t); });
  for (auto& th : ts) th.join();
}

int bits_for(int64_t v) {
  int b = 0;
  while ((int64_t{1} << b) <= v) ++b;
  return b;
}

// Build the pair list of a product Out = X * Y on known patterns: output block
// (row, col) collects every (k, q) with X_{row, x_ci[k]} and Y_{x_ci[k], col} stored,
// where q indexes Y's row x_ci[k].  Codes store (k - x_rp[row], q - y_rp[x_ci[k]]).
// Entries of one output are ordered by k then q.
void build_pairs(int32_t nrows, int32_t ncols, const std::vector<int32_t>& x_rp, const std::vector<int32_t>& x_ci,
                 const std::vector<int32_t>& y_rp, const std::vector<int32_t>& y_ci, const std::vector<int32_t>& o_rp,
                 const std::vector<int32_t>& o_ci, bool allow_byte, PairList& out) {
  const int nth = std::max(1, std::min<int>(16, static_cast<int>(std::thread::hardware_concurrency())));
  const size_t nout = o_ci.size();
  std::vector<int32_t> cnt(nout + 1, 0);
  std::vector<int64_t> max_hi(nth, 0), max_lo(nth, 0);
  std::vector<std::vector<int32_t>> pos(nth), tag(nth);
  // pass 1: counts and ranges (contributions to columns outside the output row are
  // skipped: the output pattern may be a subset of the product pattern)
  parallel_rows(nrows, [&](int32_t r0, int32_t r1, int tid) {
    auto& ps = pos[tid];
    auto& tg = tag[tid];
    ps.assign(static_cast<size_t>(ncols), -1);
    tg.assign(static_cast<size_t>(ncols), -1);
    for (int32_t r = r0; r < r1; ++r) {
      for (int32_t sidx = o_rp[r]; sidx < o_rp[r + 1]; ++sidx) { ps[o_ci[sidx]] = sidx; tg[o_ci[sidx]] = r; }
      for (int32_t k = x_rp[r]; k < x_rp[r + 1]; ++k) {
        const int32_t j = x_ci[k];
        for (int32_t q = y_rp[j]; q < y_rp[j + 1]; ++q) {
          if (tg[y_ci[q]] != r) continue;
          cnt[ps[y_ci[q]] + 1]++;
          max_hi[tid] = std::max<int64_t>(max_hi[tid], k - x_rp[r]);
          max_lo[tid] = std::max<int64_t>(max_lo[tid], q - y_rp[j]);
        }
      }
    }
  });
  int64_t mh = 0, ml = 0;
  for (int t = 0; t < nth; ++t) { mh = std::max(mh, max_hi[t]); ml = std::max(ml, max_lo[t]); }
  const int bh = bits_for(mh), bl = bits_for(ml);
  int width;
  if (allow_byte && bh + bl <= 8) width = 1;
  else if (bh + bl <= 16) width = 2;
  else if (bh + bl <= 32) width = 4;
  else { out.width = 0; return; }
  std::vector<int32_t> ptr(nout + 1, 0);
  for (size_t sidx = 0; sidx < nout; ++sidx) {
    BLK_REQUIRE(static_cast<int64_t>(ptr[sidx]) + cnt[sidx + 1] <= INT32_MAX, BLKAMG_EINVAL, "pair list too long");
    ptr[sidx + 1] = ptr[sidx] + cnt[sidx + 1];
  }
  std::vector<uint8_t> codes(static_cast<size_t>(ptr[nout]) * width);
  // pass 2: fill (each row writes only its own output range)
  parallel_rows(nrows, [&](int32_t r0, int32_t r1, int tid) {
    auto& ps = pos[tid];
    auto& tg = tag[tid];
    std::fill(tg.begin(), tg.end(), -1);
    std::vector<int32_t> cur;
    for (int32_t r = r0; r < r1; ++r) {
      const int32_t s0 = o_rp[r], s1 = o_rp[r + 1];
      cur.assign(ptr.begin() + s0, ptr.begin() + s1);
      for (int32_t sidx = s0; sidx < s1; ++sidx) { ps[o_ci[sidx]] = sidx; tg[o_ci[sidx]] = r; }
      for (int32_t k = x_rp[r]; k < x_rp[r + 1]; ++k) {
        const int32_t j = x_ci[k];
        for (int32_t q = y_rp[j]; q < y_rp[j + 1]; ++q) {
          if (tg[y_ci[q]] != r) continue;
          const uint32_t code = (static_cast<uint32_t>(k - x_rp[r]) << bl) | static_cast<uint32_t>(q - y_rp[j]);
          const int32_t at = cur[ps[y_ci[q]] - s0]++;
          std::memcpy(&codes[static_cast<size_t>(at) * width], &code, width);  // little endian
        }
      }
    }
  });
  out.width = width;
  out.shift = bl;
  upload(out.ptr, ptr);
  upload(out.codes, codes);
}

// Inside every group of `per` (<= 256) consecutive output blocks, the block offsets
// ordered by descending number of contributions (stable).
std::vector<uint8_t> count_order(const std::vector<int32_t>& ptr, int per) {
  const int64_t n = static_cast<int64_t>(ptr.size()) - 1;
  std::vector<uint8_t> out(static_cast<size_t>(n));
  std::vector<int> idx;
  for (int64_t g = 0; g < n; g += per) {
    const int m = static_cast<int>(std::min<int64_t>(per, n - g));
    idx.resize(m);
    for (int t = 0; t < m; ++t) idx[t] = t;
    std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) {
      return (ptr[g + a + 1] - ptr[g + a]) > (ptr[g + b + 1] - ptr[g + b]);
    });
    for (int t = 0; t < m; ++t) out[g + t] = static_cast<uint8_t>(idx[t]);
  }
  return out;
}

std::vector<uint8_t> identity_order(size_t n, int per) {
  std::vector<uint8_t> out(n);
  for (size_t t = 0; t < n; ++t) out[t] = static_cast<uint8_t>(t % per);
  return out;
}

// Row of the first output block of every group of `per` consecutive blocks.
std::vector<int32_t> first_rows(const std::vector<int32_t>& rp, int per) {
  const int64_t nnz = rp.back();
  std::vector<int32_t> out(static_cast<size_t>((nnz + per - 1) / per) + 1, 0);
  int32_t row = 0;
  const int32_t nr = static_cast<int32_t>(rp.size()) - 1;
  for (size_t w = 0; w + 1 < out.size(); ++w) {
    const int64_t s0 = static_cast<int64_t>(w) * per;
    while (row < nr && rp[row + 1] <= s0) ++row;
    out[w] = row;
  }
  out.back() = std::max(nr - 1, 0);  // bound for the last group
  return out;
}

// Tuning switches of the numeric plan (environment BLKAMG_PTAP_TUNE, default "ap_sort";
// flags ap_sort / c_sort / ap_nl1 / c_nl1 / c_nl3 / ap_novec / c_novec / nostage /
// ap_xcd[=C] / c_xcd[=C]).
struct PtapTune {
  std::string tn;
  bool has(const char* f) const { return tn.find(f) != std::string::npos; }
  int chunk_of(const char* key, int dflt) const {
    const size_t at = tn.find(key);
    if (at == std::string::npos) return dflt;
    const char* v = tn.c_str() + at + std::strlen(key);
    return *v == '=' ? std::max(0, std::atoi(v + 1)) : -1;
  }
};

// Plan settings that do not depend on the patterns.
void plan_settings(PtapPlan& pl, const bsr_s* A, const PtapTune& t) {
  // Measured at 128^3: three lanes per block shorten every A P pass (FP64 fine level
  // 8.0 -> 5.6 ms) and the 6x6 R AP passes; the fine FP32 R AP pass is faster with
  // one lane per block (2.1 vs 2.3 ms).
  // workgroup order: the hardware's round-robin over XCDs by default (measured at 128^3:
  // 4-6 % faster for the fine passes than XCD-contiguous ranges, whose eight separate
  // working sets overflow the shared MALL); ap_xcd / c_xcd switch back
  // (ap_xcd / c_xcd: XCD-contiguous ranges; ap_xcd=C / c_xcd=C: chunks of C; measured at
  // 128^3, runs of 32 (A P) and 8 (R AP) workgroups per XCD are 1-3 % faster again than
  // the hardware order)
  pl.ap_xcd = t.chunk_of("ap_xcd", 32);
  pl.c_xcd = t.chunk_of("c_xcd", 8);
  pl.ap_nl = t.has("ap_nl1") ? 1 : 3;
  pl.c_nl = t.has("c_nl1") ? 1 : t.has("c_nl3") ? 3 : (A->dtype == BLKAMG_F32 && A->br == 3 ? 1 : 3);
  pl.ap_vec = !t.has("ap_novec");
  pl.c_vec = !t.has("c_novec");
}

}  // namespace

}  // namespace blk

using namespace blk;

extern "C" {

int ptap_symbolic(bsr_t A, bsr_t P, bsr_t* C, void* stream) { return ptap_symbolic_ex(A, P, 0, C, stream); }

int ptap_symbolic_ex(bsr_t A, bsr_t P, int flags, bsr_t* C, void* stream) {
  BLK_API_BEGIN
  BLK_REQUIRE((flags & ~(BLKAMG_PTAP_SYMMETRIC | BLKAMG_PTAP_HOST_SYMBOLIC)) == 0, BLKAMG_EINVAL,
              "unknown ptap flags");
  BLK_REQUIRE(A != nullptr && P != nullptr && C != nullptr, BLKAMG_EINVAL, "NULL argument");
  *C = nullptr;
  BLK_REQUIRE(A->br == A->bc && A->br == P->br, BLKAMG_EINVAL, "A must be square-blocked with bs = P.bs_r");
  BLK_REQUIRE(A->nbr == A->nbc && A->nbr == P->nbr, BLKAMG_EINVAL, "A and P shapes do not match");
  BLK_REQUIRE((A->br == 3 && P->bc == 6) || (A->br == 6 && P->bc == 6), BLKAMG_EINVAL,
              "supported block shapes: A 3x3 with P 3x6, A 6x6 with P 6x6");
  BLK_REQUIRE((A->dtype == BLKAMG_F64 && P->dtype == BLKAMG_F64) ||
                  (A->dtype == BLKAMG_F32 && (P->dtype == BLKAMG_F32 || P->dtype == BLKAMG_BF16)),
              BLKAMG_EINVAL, "dtype combination must be F64/F64, F32/F32 or F32/BF16");
  hipStream_t s = as_stream(stream);
  HIP_CHECK(hipStreamSynchronize(s));
  const char* tune = std::getenv("BLKAMG_PTAP_TUNE");
  const PtapTune tn{tune ? tune : "ap_sort"};
  const bool search = std::getenv("BLKAMG_PTAP_SEARCH") != nullptr;
  const size_t acc_size = A->dtype == BLKAMG_F64 ? 8 : 4;
  ensure_host_pattern(P);
  bsr_s* R = transpose_of(P, s);
  if (!search && !(flags & BLKAMG_PTAP_HOST_SYMBOLIC) && !tn.has("host_symbolic")) {
    auto plan = std::make_shared<PtapPlan>();
    plan->A = A;
    plan->P = P;
    plan->a_nnzb = A->nnzb;
    plan->p_nnzb = P->nnzb;
    plan->n_ap_rows = A->nbr;
    plan->sym = (flags & BLKAMG_PTAP_SYMMETRIC) != 0;
    plan_settings(*plan, A, tn);
    DevBuf<int32_t> crp, cci;
    int64_t cnnz = 0;
    if (ptap_symbolic_device(A, P, R, *plan, tn.has("ap_sort"), tn.has("c_sort"), crp, cci, cnnz, s)) {
      BLK_REQUIRE(cnnz <= INT32_MAX, BLKAMG_EINVAL, "coarse pattern too large");
      plan->g_ap = pick_lanes(A->nbr ? static_cast<double>(plan->ap_nslots) / A->nbr : 0.0);
      plan->g_c = pick_lanes(P->nbc ? static_cast<double>(cnnz) / P->nbc : 0.0);
      plan->ap_val.alloc(static_cast<size_t>(plan->ap_nslots) * P->br * P->bc * acc_size);
      if (tn.has("nostage")) plan->ap_cap = plan->c_cap = 1;
      auto Cm = make_owned_device(P->nbc, P->nbc, P->bc, P->bc, A->dtype, std::move(crp), std::move(cci), cnnz, s);
      Cm->ext = plan;
      *C = Cm.release();
      return BLKAMG_OK;
    }
  }
  // host build
  ensure_host_pattern(A);
  auto plan = std::make_shared<PtapPlan>();
  std::vector<int32_t> aprp, apci, crp, cci;
  structural_product_host(A->nbr, A->h_rowptr, A->h_colidx, P->nbc, P->h_rowptr, P->h_colidx, aprp, apci);
  structural_product_host(R->nbr, R->h_rowptr, R->h_colidx, P->nbc, aprp, apci, crp, cci);
  plan->A = A;
  plan->P = P;
  plan->a_nnzb = A->nnzb;
  plan->p_nnzb = P->nnzb;
  plan->n_ap_rows = A->nbr;
  plan->g_ap = pick_lanes(A->nbr ? static_cast<double>(apci.size()) / A->nbr : 0.0);
  plan->g_c = pick_lanes(P->nbc ? static_cast<double>(cci.size()) / P->nbc : 0.0);
  plan->ap_val.alloc(apci.size() * static_cast<size_t>(P->br) * P->bc * acc_size);
  upload(plan->ap_rowptr, aprp);
  upload(plan->ap_colidx, apci);
  if (!search) {
    build_pairs(A->nbr, P->nbc, A->h_rowptr, A->h_colidx, P->h_rowptr, P->h_colidx, aprp, apci, true, plan->ap_pairs);
    plan->sym = (flags & BLKAMG_PTAP_SYMMETRIC) != 0;
    std::vector<int32_t> orp = crp, oci = cci;  // output blocks of the R*AP pass
    if (plan->sym) {
      // upper blocks (column >= row), their index in C and the index of the mirror
      std::vector<int32_t> uidx, mir;
      orp.assign(crp.size(), 0);
      oci.clear();
      for (int32_t a = 0; a + 1 < static_cast<int32_t>(crp.size()); ++a) {
        for (int32_t t = crp[a]; t < crp[a + 1]; ++t) {
          const int32_t c = cci[t];
          if (c < a) continue;
          int32_t m = -1;
          if (c != a) {
            const auto b0 = cci.begin() + crp[c], b1 = cci.begin() + crp[c + 1];
            const auto it = std::lower_bound(b0, b1, a);
            BLK_REQUIRE(it != b1 && *it == a, BLKAMG_EINVAL, "coarse pattern is not symmetric");
            m = static_cast<int32_t>(it - cci.begin());
          }
          oci.push_back(c);
          uidx.push_back(t);
          mir.push_back(m);
        }
        orp[a + 1] = static_cast<int32_t>(oci.size());
      }
      plan->c_nslots = static_cast<int64_t>(oci.size());
      upload(plan->c_up_rp, orp);
      upload(plan->c_up_idx, uidx);
      upload(plan->c_mirror, mir);
    }
    build_pairs(R->nbr, P->nbc, R->h_rowptr, R->h_colidx, aprp, apci, orp, oci, true, plan->c_pairs);
    if (!plan->c_pairs.width) plan->sym = false;  // the searching kernel computes every block
    plan->ap_nslots = static_cast<int64_t>(apci.size());
    plan_settings(*plan, A, tn);
    const int ap_spw = kBlock / plan->ap_nl, c_spw = kBlock / plan->c_nl;
    const std::vector<int32_t> ap_w = first_rows(aprp, ap_spw), c_w = first_rows(orp, c_spw);
    upload(plan->ap_slot_row0, ap_w);
    upload(plan->c_slot_row0, c_w);
    // LDS capacity: the X extent that 99.5% of the workgroups fit in (the rest read
    // from global memory), within kLdsBytes; a larger allocation for a few outliers
    // would cost resident workgroups everywhere (measured for FP64 A P at 128^3)
    auto cap_of = [](const std::vector<int32_t>& w, const std::vector<int32_t>& xrp, int nrows, size_t per) {
      std::vector<int32_t> nk;
      for (size_t g = 0; g + 1 < w.size(); ++g) {
        const int r0 = w[g], r1 = std::min(nrows - 1, w[g + 1]);
        if (r1 - r0 + 1 > kMaxR) continue;
        nk.push_back(xrp[r1 + 1] - xrp[r0]);
      }
      int cap = 1;
      if (!nk.empty()) {
        const size_t q = std::min(nk.size() - 1, (nk.size() * 995) / 1000);
        std::nth_element(nk.begin(), nk.begin() + q, nk.end());
        cap = nk[q];
      }
      const int lim = static_cast<int>((kLdsBytes - 16) / per);
      return std::max(1, std::min(cap, lim));
    };
    plan->ap_cap = cap_of(ap_w, A->h_rowptr, A->nbr, 4 + static_cast<size_t>(A->br) * A->br * dtype_size(A->dtype));
    plan->c_cap = cap_of(c_w, R->h_rowptr, R->nbr, 4);
    if (tn.has("nostage")) plan->ap_cap = plan->c_cap = 1;  // every workgroup takes the global-memory path
    if (plan->ap_pairs.width) {
      std::vector<int32_t> hp = download(plan->ap_pairs.ptr.p, plan->ap_pairs.ptr.n);
      upload(plan->ap_perm, tn.has("ap_sort") ? count_order(hp, ap_spw) : identity_order(hp.size() - 1, ap_spw));
    }
    if (plan->c_pairs.width) {
      std::vector<int32_t> hp = download(plan->c_pairs.ptr.p, plan->c_pairs.ptr.n);
      upload(plan->c_perm, tn.has("c_sort") ? count_order(hp, c_spw) : identity_order(hp.size() - 1, c_spw));
    }
  }
  auto Cm = make_owned(P->nbc, P->nbc, P->bc, P->bc, A->dtype, std::move(crp), std::move(cci));
  Cm->ext = plan;
  HIP_CHECK(hipStreamSynchronize(s));
  *C = Cm.release();
  BLK_API_END
}

int ptap_numeric(bsr_t A, bsr_t P, bsr_t C, void* stream) {
  BLK_API_BEGIN
  BLK_REQUIRE(A != nullptr && P != nullptr && C != nullptr, BLKAMG_EINVAL, "NULL argument");
  auto* pl = static_cast<PtapPlan*>(C->ext.get());
  BLK_REQUIRE(pl != nullptr, BLKAMG_EINVAL, "C was not created by ptap_symbolic");
  BLK_REQUIRE(pl->A == A && pl->P == P, BLKAMG_EINVAL, "C was created for a different (A, P)");
  BLK_REQUIRE(pl->a_nnzb == A->nnzb && pl->p_nnzb == P->nnzb, BLKAMG_ESTATE,
              "pattern of A or P changed since ptap_symbolic");
  hipStream_t s = as_stream(stream);
  bsr_s* R = transpose_of(P, s);  // refreshes R values only if P's stamp moved
  if (A->br == 3)
    numeric_shape<3, 6>(*pl, A, P, R, C, s);
  else
    numeric_shape<6, 6>(*pl, A, P, R, C, s);
  C->stamp++;
  BLK_API_END
}

int ptap_plan_info(bsr_t C, int64_t* ap_nnzb, int64_t* ap_pairs, int64_t* c_pairs, int32_t* symmetric) {
  BLK_API_BEGIN
  BLK_REQUIRE(C != nullptr, BLKAMG_EINVAL, "C is NULL");
  auto* pl = static_cast<PtapPlan*>(C->ext.get());
  BLK_REQUIRE(pl != nullptr, BLKAMG_EINVAL, "C was not created by ptap_symbolic");
  auto total = [](const PairList& L) -> int64_t {
    if (L.width == 0 || L.ptr.n == 0) return -1;
    int32_t v = 0;
    HIP_CHECK(hipMemcpy(&v, L.ptr.p + (L.ptr.n - 1), sizeof(int32_t), hipMemcpyDeviceToHost));
    return v;
  };
  if (ap_nnzb) *ap_nnzb = pl->ap_nslots;
  if (ap_pairs) *ap_pairs = total(pl->ap_pairs);
  if (c_pairs) *c_pairs = total(pl->c_pairs);
  if (symmetric) *symmetric = pl->sym ? 1 : 0;
  BLK_API_END
}

}  // extern "C"

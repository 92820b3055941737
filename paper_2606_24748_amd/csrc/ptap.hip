// Galerkin coarse operator A_c = P^T A P on a fixed block pattern (paper §2.1,
// §3.1, §3.5).  The symbolic phase (host) builds the pattern of A P and of A_c and
// keeps it; the numeric phase is device-only, allocation-free and deterministic:
//   pass 1: AP_ib = sum_j A_ij P_jb          (one lane per output block of AP)
//   pass 2: C_ac  = sum_i R_ai AP_ic, R = P^T (one lane per output block of C)
// The transpose R comes from P's value-stamped cache, so a recompute with an
// unchanged prolongator never rebuilds prolongator-side data (paper §3.5).
#include <algorithm>

#include "spmv_core.hpp"

namespace blk {

struct PtapPlan {
  const bsr_s* A = nullptr;
  const bsr_s* P = nullptr;
  int64_t a_nnzb = 0, p_nnzb = 0;
  int32_t n_ap_rows = 0;
  DevBuf<int32_t> ap_rowptr, ap_colidx;
  DevBuf<char> ap_val;  // scratch for A P in the accumulation type
  int g_ap = 32, g_c = 32;
};

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

template <int BR, int BC, class TA_, class TP, class TA>
void run_numeric(const PtapPlan& pl, const bsr_s* A, const bsr_s* P, const bsr_s* R, bsr_s* C, hipStream_t s) {
  TA* ap = reinterpret_cast<TA*>(pl.ap_val.p);
  if (A->nbr > 0) {
#define BLK_AP(GG)                                                                                      \
  ap_kernel<BR, BC, GG, TA_, TP, TA><<<grid_for(GG, A->nbr), kBlock, 0, s>>>(                            \
      A->nbr, A->rowptr, A->colidx, static_cast<const TA_*>(A->val), P->rowptr, P->colidx,               \
      static_cast<const TP*>(P->val), pl.ap_rowptr.p, pl.ap_colidx.p, ap)
    if (pl.g_ap == 16) BLK_AP(16); else BLK_AP(32);
#undef BLK_AP
    HIP_CHECK(hipGetLastError());
  }
  if (C->nbr > 0) {
#define BLK_RAP(GG)                                                                                     \
  rap_kernel<BR, BC, GG, TP, TA, TA_><<<grid_for(GG, C->nbr), kBlock, 0, s>>>(                           \
      C->nbr, R->rowptr, R->colidx, static_cast<const TP*>(R->val), pl.ap_rowptr.p, pl.ap_colidx.p, ap,  \
      C->rowptr, C->colidx, static_cast<TA_*>(C->val))
    if (pl.g_c == 16) BLK_RAP(16); else BLK_RAP(32);
#undef BLK_RAP
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

}  // namespace blk

using namespace blk;

extern "C" {

int ptap_symbolic(bsr_t A, bsr_t P, bsr_t* C, void* stream) {
  BLK_API_BEGIN
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
  ensure_host_pattern(A);
  ensure_host_pattern(P);
  bsr_s* R = transpose_of(P, s);
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
  const size_t acc_size = A->dtype == BLKAMG_F64 ? 8 : 4;
  plan->ap_val.alloc(apci.size() * static_cast<size_t>(P->br) * P->bc * acc_size);
  upload(plan->ap_rowptr, aprp);
  upload(plan->ap_colidx, apci);
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

}  // extern "C"

// Plan of the numeric Galerkin product A_c = P^T A P (paper §3.1, §3.5): the patterns
// of A P and of A_c, the per-output contribution lists and the workgroup tables of
// the numeric kernels.  Built once by ptap_symbolic (on the device, or on the host),
// read by every ptap_numeric.
#pragma once

#include <vector>

#include "internal.hpp"

namespace blk {

constexpr int kMaxR = 48;         // rows of a workgroup whose tables are staged in LDS
constexpr int kLdsBytes = 49152;  // LDS of a numeric workgroup at most

// Contributions to one output block, listed once at symbolic time: each entry packs
// (index within the first operand's row, index within the second operand's row)
// into `width` bytes, high part shifted left by `shift`.
struct PairList {
  DevBuf<uint8_t> codes;
  DevBuf<int32_t> ptr;  // ptr[s]..ptr[s+1]: entries of output block s
  int width = 0;        // 1, 2 or 4 bytes; 0 = not built (use the searching kernels)
  int shift = 0;
};

struct PtapPlan {
  const bsr_s* A = nullptr;
  const bsr_s* P = nullptr;
  int64_t a_nnzb = 0, p_nnzb = 0;
  int32_t n_ap_rows = 0;
  DevBuf<int32_t> ap_rowptr, ap_colidx;
  DevBuf<char> ap_val;  // scratch for A P in the accumulation type
  int g_ap = 32, g_c = 32;
  PairList ap_pairs;    // per AP block: (block of A row i, block of P row j)
  PairList c_pairs;     // per C block: (entry of R row a, block of AP row i)
  int64_t ap_nslots = 0;
  DevBuf<int32_t> ap_slot_row0, c_slot_row0;  // row of the first block of each workgroup
  DevBuf<uint8_t> ap_perm, c_perm;             // per workgroup: order in which lanes take the blocks
  int ap_cap = 0, c_cap = 0;                   // LDS capacity (entries of X rows) of a workgroup
  int ap_nl = 1, c_nl = 1;                     // lanes per output block (1 or 3)
  int ap_xcd = 32, c_xcd = 8;                  // workgroup order: 0 hardware, -1 XCD-contiguous, C > 0 chunks
  bool ap_vec = true, c_vec = true;
  // symmetric mode: only blocks with column >= row are computed (upper list), each
  // off-diagonal one is also stored transposed at its mirror position
  bool sym = false;
  int64_t c_nslots = 0;
  DevBuf<int32_t> c_up_rp, c_up_idx, c_mirror;
};

// The plan's product patterns, contribution lists and workgroup tables built on the
// device (same contents as the host build).  Fills plan->ap_rowptr / ap_colidx /
// ap_pairs / c_pairs / c_up_* / *_slot_row0 / *_perm / *_cap / ap_nslots / c_nslots
// and the coarse pattern (c_rowptr, c_colidx on the device, c_nnzb).  plan->sym,
// ap_nl and c_nl must be set.  Returns false, with nothing usable built, when a row
// offset does not fit 16 bits (the caller then builds on the host).  EINVAL when sym
// is set and the coarse pattern is not symmetric.  Sync.
bool ptap_symbolic_device(const bsr_s* A, const bsr_s* P, const bsr_s* R, PtapPlan& plan, bool ap_sort,
                          bool c_sort, DevBuf<int32_t>& c_rowptr, DevBuf<int32_t>& c_colidx, int64_t& c_nnzb,
                          hipStream_t s);

}  // namespace blk

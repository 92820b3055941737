// Internal object definitions shared by the translation units of libblkamg.
#pragma once

#include "common.hpp"

struct bsr_s;

namespace blk {

// Cached explicit transpose R = A^T (pattern built once on the host; values
// refreshed on the device whenever the owner's value stamp moved).
struct TransposeCache {
  DevBuf<int32_t> rowptr, colidx, map;  // map[t] = block of A copied (transposed) into R block t
  DevBuf<char> val;
  uint64_t stamp = 0;                   // owner stamp the values were copied at (0 = never)
  std::unique_ptr<bsr_s> R;             // view over the arrays above
};

}  // namespace blk

struct bsr_s {
  int32_t nbr = 0, nbc = 0, br = 0, bc = 0;
  int64_t nnzb = 0;
  int dtype = BLKAMG_F64;
  const int32_t* rowptr = nullptr;
  const int32_t* colidx = nullptr;
  void* val = nullptr;
  // owned storage (library-created matrices)
  blk::DevBuf<int32_t> own_rowptr, own_colidx;
  blk::DevBuf<char> own_val;
  uint64_t stamp = 1;  // value-state stamp
  int tuned[2] = {0, 0};  // autotuned SpMV lane code for 1 and for 8 right-hand sides (0 = heuristic)
  std::unique_ptr<blk::TransposeCache> tcache;
  // symmetric reads: mirror position of every strictly lower block (built once, on the
  // device; sym_state 0 = not built, 1 = built, -1 = pattern not symmetric)
  blk::DevBuf<int32_t> sym_mir;
  int sym_state = 0;
  int sym_dist = 0;  // median over rows of the distance to the row's first lower column
  // FP32 copy of the values that a mixed-precision hierarchy keeps as its level-0
  // operator (same pattern): coo_assemble_blocked writes it beside the values, and
  // f32_copy_stamp is the stamp it then matches (the hierarchy casts otherwise)
  bsr_s* f32_copy = nullptr;
  uint64_t f32_copy_stamp = 0;
  // host copy of the pattern (filled on demand or at creation)
  std::vector<int32_t> h_rowptr, h_colidx;
  bool h_pattern = false;
  // plan attached by ptap_symbolic to the coarse matrix it creates
  std::shared_ptr<void> ext;

  size_t block_elems() const { return static_cast<size_t>(br) * bc; }
  size_t val_bytes() const { return static_cast<size_t>(nnzb) * block_elems() * blk::dtype_size(dtype); }
  double avg_blocks_per_row() const { return nbr ? static_cast<double>(nnzb) / nbr : 0.0; }
};

namespace blk {

// Library-owned matrix with the given host pattern (uploaded) and zeroed values.
std::unique_ptr<bsr_s> make_owned(int32_t nbr, int32_t nbc, int32_t br, int32_t bc, int dtype,
                                  std::vector<int32_t> h_rowptr, std::vector<int32_t> h_colidx);
// Library-owned matrix over device pattern arrays (taken over) and zeroed values; its
// host pattern is downloaded on demand.  Sync.
std::unique_ptr<bsr_s> make_owned_device(int32_t nbr, int32_t nbc, int32_t br, int32_t bc, int dtype,
                                         DevBuf<int32_t>&& d_rowptr, DevBuf<int32_t>&& d_colidx, int64_t nnzb,
                                         hipStream_t s);
// Make sure A->h_rowptr / h_colidx hold the pattern (downloads once; sync).
void ensure_host_pattern(bsr_s* A);
// Transpose cache of A, built if needed; values refreshed on `s` if stale.
bsr_s* transpose_of(bsr_s* A, hipStream_t s);
// Mirror index of A's strictly lower blocks for the symmetric SpMV reads (position
// of block (colidx[k], row) for every block k with colidx[k] < row), built once on
// the device; nullptr when A is not square-blocked or its pattern is not symmetric.
// Sync on the first call.
const int32_t* symmetric_mirror(bsr_s* A, hipStream_t s);
// y = alpha op(A) x + beta y
// (code != 0 forces that lane configuration)
// (mir: symmetric reads with that mirror index, one right-hand side; see row_product)
void spmv(const bsr_s* A, double alpha, const void* x, double beta, void* y, int vdt, int nrhs,
          hipStream_t s, int code = 0, const int32_t* mir = nullptr, int sym_dist = 0);
// SpMV lane configuration (G * 8 + U) for A with nrhs right-hand sides: the
// autotuned one if present, else a heuristic on the mean blocks per row.
int lanes_for(const bsr_s* A, int nrhs = 1);
// The lane configuration for A's SpMV with or without symmetric reads (mir).
int lanes_for_reads(const bsr_s* A, int nrhs, const int32_t* mir);
// Time every compiled lane configuration of y = A x (vectors of dtype vdt, nrhs
// columns) with device events and keep the fastest in A; returns its code.  Sync.
int autotune_lanes(bsr_s* A, int vdt, int nrhs, hipStream_t s);
// Structural product of two host block patterns (sorted rows, no dropping).
void structural_product_host(int32_t nra, const std::vector<int32_t>& rpa, const std::vector<int32_t>& cia,
                             int32_t ncb, const std::vector<int32_t>& rpb, const std::vector<int32_t>& cib,
                             std::vector<int32_t>& rpc, std::vector<int32_t>& cic);
// Structural product of two device patterns (sorted unique columns per row; Y has
// ncols columns), built on the device; false when a row of X is longer than 65536
// entries or a row of Y longer than 65536 (nothing built).  Sync.
bool structural_product_device(int32_t nrows, int32_t ncols, const int32_t* x_rp, const int32_t* x_ci,
                               const int32_t* y_rp, const int32_t* y_ci, DevBuf<int32_t>& out_rp,
                               DevBuf<int32_t>& out_ci, int64_t& nnz, hipStream_t s);
// Cast a value array between dtypes on the device.
void cast_values(const void* src, int sdt, void* dst, int ddt, size_t n, hipStream_t s);
// Tentative prolongator rows and coarse near-null space on the device (per-aggregate
// Householder QR); false if an aggregate is too large for it (nothing computed).
void rigid_body_modes_device(int32_t n, const double* d_coords, double* d_B, hipStream_t s);
bool tentative_device(int32_t nbr, int32_t bs, const int32_t* d_agg, int32_t n_agg, const double* d_B, double* d_Pt,
                      double* d_Bc, hipStream_t s);

}  // namespace blk

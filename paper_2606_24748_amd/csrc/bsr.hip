// Rectangular-block sparse matrix handle, SpMV and SpMV-transpose (paper §2.3, §4.2),
// and the C-ABI error plumbing.
#include <cstdio>
#include <cstdlib>

#include "spmv_core.hpp"

namespace blk {

namespace {
thread_local std::string g_last_error;
}

void set_last_error(const std::string& msg) { g_last_error = msg; }

hipStream_t as_stream(void* s) { return static_cast<hipStream_t>(s); }

int num_cus() {
  static int n = 0;
  if (n == 0) {
    int dev = 0;
    int v = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0)
      n = v;
    else
      n = 256;
  }
  return n;
}

std::unique_ptr<bsr_s> make_owned(int32_t nbr, int32_t nbc, int32_t br, int32_t bc, int dtype,
                                  std::vector<int32_t> h_rowptr, std::vector<int32_t> h_colidx) {
  auto A = std::make_unique<bsr_s>();
  A->nbr = nbr;
  A->nbc = nbc;
  A->br = br;
  A->bc = bc;
  A->dtype = dtype;
  A->nnzb = static_cast<int64_t>(h_colidx.size());
  upload(A->own_rowptr, h_rowptr);
  upload(A->own_colidx, h_colidx);
  A->own_val.alloc(std::max<size_t>(A->val_bytes(), 0));
  if (A->own_val.p) HIP_CHECK(hipMemset(A->own_val.p, 0, A->val_bytes()));
  A->rowptr = A->own_rowptr.p;
  A->colidx = A->own_colidx.p;
  A->val = A->own_val.p;
  A->h_rowptr = std::move(h_rowptr);
  A->h_colidx = std::move(h_colidx);
  A->h_pattern = true;
  return A;
}

std::unique_ptr<bsr_s> make_owned_device(int32_t nbr, int32_t nbc, int32_t br, int32_t bc, int dtype,
                                         DevBuf<int32_t>&& d_rowptr, DevBuf<int32_t>&& d_colidx, int64_t nnzb,
                                         hipStream_t s) {
  auto A = std::make_unique<bsr_s>();
  A->nbr = nbr;
  A->nbc = nbc;
  A->br = br;
  A->bc = bc;
  A->dtype = dtype;
  A->nnzb = nnzb;
  A->own_rowptr = std::move(d_rowptr);
  A->own_colidx = std::move(d_colidx);
  A->own_val.alloc(A->val_bytes());
  if (A->own_val.p) HIP_CHECK(hipMemsetAsync(A->own_val.p, 0, A->val_bytes(), s));
  HIP_CHECK(hipStreamSynchronize(s));
  A->rowptr = A->own_rowptr.p;
  A->colidx = A->own_colidx.p;
  A->val = A->own_val.p;
  A->h_pattern = false;  // downloaded on demand
  return A;
}

void ensure_host_pattern(bsr_s* A) {
  if (A->h_pattern) return;
  A->h_rowptr = download(A->rowptr, static_cast<size_t>(A->nbr) + 1);
  A->h_colidx = download(A->colidx, static_cast<size_t>(A->nnzb));
  A->h_pattern = true;
}

// (G, U) for a matrix: G lanes per block row, U blocks per lane per step.  The
// heuristic targets about one step per row with enough bytes in flight per wave;
// BLKAMG_SPMV_LANES="GxU" overrides it (experiments).
int lanes_for(const bsr_s* A, int nrhs) {
  static int forced = -1;
  if (forced < 0) {
    forced = 0;
    if (const char* e = std::getenv("BLKAMG_SPMV_LANES")) {
      int g = 0, u = 0;
      if (std::sscanf(e, "%dx%d", &g, &u) == 2) forced = g * 8 + u;
    }
  }
  if (forced > 0) return forced;
  if (const int t = A->tuned[nrhs > 1 ? 1 : 0]) return t;
  const double avg = A->avg_blocks_per_row();
  const size_t vb = A->block_elems() * dtype_size(A->dtype);  // bytes per block
  // Measured on the 128^3 hierarchy.  Fine 3x3 operator (27 blocks per row): 32 lanes,
  // one block per lane, for both F32 and F64.  6x6 F64 blocks (288 bytes) want two
  // blocks per lane and fewer lanes (level-1 operator, 26 per row: 16 x 2 112 us against
  // 188 us with 32 x 1; its prolongator, 4.5 per row: 8 x 2 21 against 32 us).  Long
  // rows of the restrictions' 6x3 and 6x6 blocks (106-121 per row) take 64 x 2 (0.289
  // against 0.304 ms for the fine F64 one, 0.153 against 0.158 ms in F32; 20 against
  // 40 us for the level-1 F64 one); long rows of 3x3 blocks (the triquadratic fine
  // operator, 62 per row) keep one block per lane.
  const bool big = vb >= 288;
  if (avg <= 8.0) return lane_code(8, big ? 2 : 1);
  if (avg <= 16.0) return lane_code(16, 1);
  if (avg <= 40.0) return big ? lane_code(16, 2) : lane_code(32, 1);
  return lane_code(64, A->block_elems() >= 18 ? 2 : 1);
}

namespace {

// ---- transpose values: R block t (bc x br) = A block map[t] transposed ----
template <class T>
__global__ void transpose_values_kernel(int64_t nnzb, int br, int bc, const int32_t* __restrict__ map,
                                        const T* __restrict__ in, T* __restrict__ out) {
  const int64_t be = static_cast<int64_t>(br) * bc;
  const int64_t total = nnzb * be;
  for (int64_t g = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; g < total;
       g += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int64_t t = g / be;
    const int e = static_cast<int>(g - t * be);
    const int jj = e / br, ii = e - jj * br;  // output element (jj, ii) of a bc x br block
    out[g] = in[static_cast<int64_t>(map[t]) * be + ii * bc + jj];
  }
}

// ---- generic fallback SpMV: one thread per output scalar ----
template <class TM, class TX, class TA>
__global__ void spmv_generic_kernel(int nbr, int br, int bc, int nrhs, const int32_t* __restrict__ rowptr,
                                    const int32_t* __restrict__ colidx, const TM* __restrict__ val,
                                    const TX* __restrict__ x, TA alpha, TA beta, TX* __restrict__ y) {
  const int64_t per_row = static_cast<int64_t>(br) * nrhs;
  const int64_t total = static_cast<int64_t>(nbr) * per_row;
  for (int64_t g = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; g < total;
       g += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int row = static_cast<int>(g / per_row);
    const int e = static_cast<int>(g - row * per_row);
    const int i = e / nrhs, q = e - i * nrhs;
    TA s = TA(0);
    for (int k = rowptr[row]; k < rowptr[row + 1]; ++k) {
      const TM* b = val + static_cast<size_t>(k) * br * bc + static_cast<size_t>(i) * bc;
      const TX* xc = x + static_cast<size_t>(colidx[k]) * bc * nrhs + q;
      for (int j = 0; j < bc; ++j) s = fmadd(ld<TA>(b + j), ld<TA>(xc + static_cast<size_t>(j) * nrhs), s);
    }
    TA v = alpha * s;
    if (beta != TA(0)) v = fmadd(beta, ld<TA>(y + g), v);
    st(y + g, v);
  }
}

template <int BR, int BC, class TM, class TX, class TA>
void spmv_fast(const bsr_s* A, TA alpha, const TX* x, TA beta, TX* y, int nrhs, hipStream_t s, int code,
               const int32_t* mir, int sym_dist) {
  const int G = code ? code : lanes_for(A, nrhs);
  const auto* v = static_cast<const TM*>(A->val);
  if (nrhs == 1) {
    launch_rows<BR, BC, 1, TM, TX, TA>(G, A->nbr, A->rowptr, A->colidx, v, x, EpiAxpby<TX, TA>{y, alpha, beta}, s,
                                       mir, sym_dist);
  } else {
    launch_rows<BR, BC, 8, TM, TX, TA>(G, A->nbr, A->rowptr, A->colidx, v, x, EpiAxpby<TX, TA>{y, alpha, beta}, s);
  }
}

template <class TM, class TX, class TA>
void spmv_typed(const bsr_s* A, TA alpha, const TX* x, TA beta, TX* y, int nrhs, hipStream_t s, int code,
                const int32_t* mir, int sym_dist) {
  if (A->nbr == 0) return;
  const int br = A->br, bc = A->bc;
  if (nrhs == 1 || nrhs == 8) {
    if (br == 3 && bc == 3) return spmv_fast<3, 3, TM, TX, TA>(A, alpha, x, beta, y, nrhs, s, code, mir, sym_dist);
    if (br == 3 && bc == 6) return spmv_fast<3, 6, TM, TX, TA>(A, alpha, x, beta, y, nrhs, s, code, nullptr, 0);
    if (br == 6 && bc == 3) return spmv_fast<6, 3, TM, TX, TA>(A, alpha, x, beta, y, nrhs, s, code, nullptr, 0);
    if (br == 6 && bc == 6) return spmv_fast<6, 6, TM, TX, TA>(A, alpha, x, beta, y, nrhs, s, code, mir, sym_dist);
  }
  const int64_t total = static_cast<int64_t>(A->nbr) * br * nrhs;
  const int grid = static_cast<int>(std::min<int64_t>((total + 255) / 256, 1 << 20));
  spmv_generic_kernel<TM, TX, TA><<<grid, 256, 0, s>>>(A->nbr, br, bc, nrhs, A->rowptr, A->colidx,
                                                       static_cast<const TM*>(A->val), x, alpha, beta, y);
  HIP_CHECK(hipGetLastError());
}

template <class TI, class TO>
__global__ void cast_kernel(const TI* __restrict__ in, TO* __restrict__ out, size_t n) {
  for (size_t g = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x; g < n;
       g += static_cast<size_t>(gridDim.x) * blockDim.x)
    out[g] = static_cast<TO>(in[g]);
}
__global__ void cast_f64_bf16_kernel(const double* __restrict__ in, bf16* __restrict__ out, size_t n) {
  for (size_t g = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x; g < n;
       g += static_cast<size_t>(gridDim.x) * blockDim.x)
    out[g] = to_bf16(static_cast<float>(in[g]));
}
__global__ void cast_f32_bf16_kernel(const float* __restrict__ in, bf16* __restrict__ out, size_t n) {
  for (size_t g = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x; g < n;
       g += static_cast<size_t>(gridDim.x) * blockDim.x)
    out[g] = to_bf16(in[g]);
}

}  // namespace

void cast_values(const void* src, int sdt, void* dst, int ddt, size_t n, hipStream_t s) {
  if (n == 0) return;
  const int grid = static_cast<int>(std::min<size_t>((n + 255) / 256, 1 << 16));
  if (sdt == ddt) {
    HIP_CHECK(hipMemcpyAsync(dst, src, n * dtype_size(sdt), hipMemcpyDeviceToDevice, s));
  } else if (sdt == BLKAMG_F64 && ddt == BLKAMG_F32) {
    cast_kernel<double, float><<<grid, 256, 0, s>>>(static_cast<const double*>(src), static_cast<float*>(dst), n);
  } else if (sdt == BLKAMG_F32 && ddt == BLKAMG_F64) {
    cast_kernel<float, double><<<grid, 256, 0, s>>>(static_cast<const float*>(src), static_cast<double*>(dst), n);
  } else if (sdt == BLKAMG_F64 && ddt == BLKAMG_BF16) {
    cast_f64_bf16_kernel<<<grid, 256, 0, s>>>(static_cast<const double*>(src), static_cast<bf16*>(dst), n);
  } else if (sdt == BLKAMG_F32 && ddt == BLKAMG_BF16) {
    cast_f32_bf16_kernel<<<grid, 256, 0, s>>>(static_cast<const float*>(src), static_cast<bf16*>(dst), n);
  } else {
    fail(BLKAMG_EINVAL, "unsupported cast");
  }
  HIP_CHECK(hipGetLastError());
}

void spmv(const bsr_s* A, double alpha, const void* x, double beta, void* y, int vdt, int nrhs, hipStream_t s,
          int code, const int32_t* mir, int sym_dist) {
  BLK_REQUIRE(nrhs >= 1 && nrhs <= 8, BLKAMG_EINVAL, "nrhs must be in 1..8");
  if (A->nbr > 0) BLK_REQUIRE(y != nullptr, BLKAMG_EINVAL, "y is NULL");
  if (A->nnzb > 0) BLK_REQUIRE(x != nullptr, BLKAMG_EINVAL, "x is NULL");
  if (A->dtype == BLKAMG_F64 && vdt == BLKAMG_F64) {
    spmv_typed<double, double, double>(A, alpha, static_cast<const double*>(x), beta, static_cast<double*>(y), nrhs, s,
                                       code, mir, sym_dist);
  } else if (A->dtype == BLKAMG_F32 && vdt == BLKAMG_F32) {
    spmv_typed<float, float, float>(A, static_cast<float>(alpha), static_cast<const float*>(x),
                                    static_cast<float>(beta), static_cast<float*>(y), nrhs, s, code, mir, sym_dist);
  } else if (A->dtype == BLKAMG_BF16 && vdt == BLKAMG_F32) {
    spmv_typed<bf16, float, float>(A, static_cast<float>(alpha), static_cast<const float*>(x),
                                   static_cast<float>(beta), static_cast<float*>(y), nrhs, s, code, mir, sym_dist);
  } else {
    fail(BLKAMG_EINVAL, "unsupported matrix/vector dtype combination");
  }
}

int autotune_lanes(bsr_s* A, int vdt, int nrhs, hipStream_t s) {
  BLK_REQUIRE(nrhs == 1 || nrhs == 8, BLKAMG_EINVAL, "autotune supports nrhs 1 or 8");
  if (A->nbr == 0 || A->nnzb == 0) return lanes_for(A, nrhs);
  const size_t vs = dtype_size(vdt == BLKAMG_F64 ? BLKAMG_F64 : BLKAMG_F32);
  DevBuf<char> x(static_cast<size_t>(A->nbc) * A->bc * nrhs * vs);
  DevBuf<char> y(static_cast<size_t>(A->nbr) * A->br * nrhs * vs);
  HIP_CHECK(hipMemsetAsync(x.p, 0, x.bytes(), s));
  hipEvent_t e0, e1;
  HIP_CHECK(hipEventCreate(&e0));
  HIP_CHECK(hipEventCreate(&e1));
  int best = 0;
  float best_ms = 0.0f;
  try {
    for (int code : kLaneCodes) {
      for (int w = 0; w < 2; ++w) spmv(A, 1.0, x.p, 0.0, y.p, vdt, nrhs, s, code);
      constexpr int kReps = 5;
      HIP_CHECK(hipEventRecord(e0, s));
      for (int r = 0; r < kReps; ++r) spmv(A, 1.0, x.p, 0.0, y.p, vdt, nrhs, s, code);
      HIP_CHECK(hipEventRecord(e1, s));
      HIP_CHECK(hipEventSynchronize(e1));
      float ms = 0.0f;
      HIP_CHECK(hipEventElapsedTime(&ms, e0, e1));
      if (best == 0 || ms < best_ms) { best = code; best_ms = ms; }
    }
  } catch (...) {
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    throw;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  A->tuned[nrhs > 1 ? 1 : 0] = best;
  return best;
}

// One thread per block row: every strictly lower block (row, c) finds its mirror
// (c, row) by binary search in row c (columns ascending); a missing mirror clears
// *ok (a row with unsorted columns can only fail the search, so every entry
// written is a valid block position).
__global__ void sym_mirror_kernel(int nbr, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                  int32_t* __restrict__ mir, int* __restrict__ ok, int32_t* __restrict__ dist) {
  const int row = blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= nbr) return;
  int far = 0;
  for (int k = rp[row]; k < rp[row + 1]; ++k) {
    const int c = ci[k];
    if (c >= row) {
      mir[k] = k;  // upper part: read in place (entry unused)
      continue;
    }
    int lo = rp[c], hi = rp[c + 1], at = -1;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      const int v = ci[mid];
      if (v == row) { at = mid; break; }
      if (v < row) lo = mid + 1; else hi = mid;
    }
    if (at < 0) *ok = 0;
    mir[k] = at < 0 ? k : at;  // a valid block position either way
    far = max(far, row - c);
  }
  dist[row] = far;
}

const int32_t* symmetric_mirror(bsr_s* A, hipStream_t s) {
  if (A->sym_state == 0) {
    A->sym_state = -1;
    if (A->br == A->bc && A->nbr == A->nbc && A->nnzb > 0) {
      A->sym_mir.alloc(static_cast<size_t>(A->nnzb));
      DevBuf<int> ok(1);
      DevBuf<int32_t> dist(static_cast<size_t>(A->nbr));
      const int one = 1;
      HIP_CHECK(hipMemcpyAsync(ok.p, &one, sizeof(int), hipMemcpyHostToDevice, s));
      sym_mirror_kernel<<<(A->nbr + 255) / 256, 256, 0, s>>>(A->nbr, A->rowptr, A->colidx, A->sym_mir.p, ok.p,
                                                              dist.p);
      HIP_CHECK(hipGetLastError());
      int h = 0;
      HIP_CHECK(hipMemcpyAsync(&h, ok.p, sizeof(int), hipMemcpyDeviceToHost, s));
      std::vector<int32_t> d = download(dist.p, dist.n, s);
      if (h) {
        A->sym_state = 1;
        std::nth_element(d.begin(), d.begin() + d.size() / 2, d.end());
        A->sym_dist = d[d.size() / 2];
      } else {
        A->sym_mir.release();
      }
    }
  }
  return A->sym_state == 1 ? A->sym_mir.p : nullptr;
}

int lanes_for_reads(const bsr_s* A, int nrhs, const int32_t* mir) {
  // symmetric reads of 3x3 blocks: 16 lanes per row, two blocks per lane and step
  // (measured on the fine FP64 operator at 128^3: 0.768 ms against 0.79-0.83 ms with
  // 32 x 1, 32 x 2, 8 x 1-2 and 1.1 ms with 64 lanes); of 6x6 F64 blocks: 8 x 2
  // (level-1 operator at 128^3: 94 us against 98 with 16 x 2 and 126 with 32 x 1)
  if (mir && nrhs == 1 && A->tuned[0] == 0) {
    if (A->br == 3) return lane_code(16, 2);
    if (A->block_elems() * dtype_size(A->dtype) >= 288) return lane_code(8, 2);
  }
  return lanes_for(A, nrhs);
}

bsr_s* transpose_of(bsr_s* A, hipStream_t s) {
  if (!A->tcache) {
    ensure_host_pattern(A);
    auto tc = std::make_unique<TransposeCache>();
    std::vector<int32_t> rp(static_cast<size_t>(A->nbc) + 1, 0), ci(static_cast<size_t>(A->nnzb)),
        mp(static_cast<size_t>(A->nnzb));
    for (int64_t k = 0; k < A->nnzb; ++k) rp[A->h_colidx[k] + 1]++;
    for (int32_t c = 0; c < A->nbc; ++c) rp[c + 1] += rp[c];
    std::vector<int32_t> next(rp.begin(), rp.end() - 1);
    for (int32_t r = 0; r < A->nbr; ++r)
      for (int32_t k = A->h_rowptr[r]; k < A->h_rowptr[r + 1]; ++k) {
        const int32_t pos = next[A->h_colidx[k]]++;
        ci[pos] = r;
        mp[pos] = k;
      }
    upload(tc->rowptr, rp);
    upload(tc->colidx, ci);
    upload(tc->map, mp);
    tc->val.alloc(A->val_bytes());
    auto R = std::make_unique<bsr_s>();
    R->nbr = A->nbc;
    R->nbc = A->nbr;
    R->br = A->bc;
    R->bc = A->br;
    R->nnzb = A->nnzb;
    R->dtype = A->dtype;
    R->rowptr = tc->rowptr.p;
    R->colidx = tc->colidx.p;
    R->val = tc->val.p;
    R->h_rowptr = std::move(rp);
    R->h_colidx = std::move(ci);
    R->h_pattern = true;
    tc->R = std::move(R);
    A->tcache = std::move(tc);
  }
  TransposeCache* tc = A->tcache.get();
  if (tc->stamp != A->stamp) {
    if (A->nnzb > 0) {
      const int64_t total = A->nnzb * static_cast<int64_t>(A->block_elems());
      const int grid = static_cast<int>(std::min<int64_t>((total + 255) / 256, 1 << 16));
      switch (A->dtype) {
        case BLKAMG_F64:
          transpose_values_kernel<double><<<grid, 256, 0, s>>>(A->nnzb, A->br, A->bc, tc->map.p,
                                                               static_cast<const double*>(A->val),
                                                               reinterpret_cast<double*>(tc->val.p));
          break;
        case BLKAMG_F32:
          transpose_values_kernel<float><<<grid, 256, 0, s>>>(A->nnzb, A->br, A->bc, tc->map.p,
                                                              static_cast<const float*>(A->val),
                                                              reinterpret_cast<float*>(tc->val.p));
          break;
        default:
          transpose_values_kernel<uint16_t><<<grid, 256, 0, s>>>(A->nnzb, A->br, A->bc, tc->map.p,
                                                                 static_cast<const uint16_t*>(A->val),
                                                                 reinterpret_cast<uint16_t*>(tc->val.p));
      }
      HIP_CHECK(hipGetLastError());
    }
    tc->stamp = A->stamp;
    tc->R->stamp++;
  }
  return tc->R.get();
}

}  // namespace blk

using namespace blk;

extern "C" {

const char* blkamg_last_error(void) { return g_last_error.c_str(); }

int blkamg_version(void) { return 100; }

int blkamg_set_allocator(blkamg_alloc_fn alloc_fn, blkamg_free_fn free_fn, void* ctx) {
  BLK_API_BEGIN
  BLK_REQUIRE((alloc_fn == nullptr) == (free_fn == nullptr), BLKAMG_EINVAL,
              "alloc_fn and free_fn must both be set or both be NULL");
  std::lock_guard<std::mutex> g(allocator_mutex());
  DeviceAllocator& a = allocator_slot();
  a.alloc_fn = alloc_fn;
  a.free_fn = free_fn;
  a.ctx = alloc_fn ? ctx : nullptr;
  BLK_API_END
}

int bsr_create(int32_t nbr, int32_t nbc, int32_t bs_r, int32_t bs_c, int64_t nnzb, const int32_t* d_rowptr,
               const int32_t* d_colidx, void* d_val, int dtype, void* stream, bsr_t* out) {
  BLK_API_BEGIN
  BLK_REQUIRE(out != nullptr, BLKAMG_EINVAL, "out is NULL");
  *out = nullptr;
  BLK_REQUIRE(nbr >= 0 && nbc >= 0 && nnzb >= 0, BLKAMG_EINVAL, "negative size");
  BLK_REQUIRE(bs_r >= 1 && bs_r <= 8 && bs_c >= 1 && bs_c <= 8, BLKAMG_EINVAL, "block size must be in 1..8");
  BLK_REQUIRE(nnzb <= INT32_MAX, BLKAMG_EINVAL, "nnzb exceeds int32 index range");
  BLK_REQUIRE(nnzb == 0 || (nbr > 0 && nbc > 0), BLKAMG_EINVAL, "blocks stored in an empty shape");
  (void)dtype_size(dtype);
  BLK_REQUIRE(d_rowptr != nullptr, BLKAMG_EINVAL, "rowptr is NULL");
  BLK_REQUIRE(nnzb == 0 || (d_colidx != nullptr && d_val != nullptr), BLKAMG_EINVAL, "colidx/val is NULL");
  auto A = std::make_unique<bsr_s>();
  A->nbr = nbr;
  A->nbc = nbc;
  A->br = bs_r;
  A->bc = bs_c;
  A->nnzb = nnzb;
  A->dtype = dtype;
  A->rowptr = d_rowptr;
  A->colidx = d_colidx;
  A->val = d_val;
  const char* v = std::getenv("BLKAMG_VALIDATE");
  if (v && v[0] == '1') {
    hipStream_t s = as_stream(stream);
    A->h_rowptr = download(A->rowptr, static_cast<size_t>(nbr) + 1, s);
    A->h_colidx = download(A->colidx, static_cast<size_t>(nnzb), s);
    A->h_pattern = true;
    BLK_REQUIRE(A->h_rowptr[0] == 0 && A->h_rowptr[nbr] == nnzb, BLKAMG_EINVAL, "rowptr ends do not match nnzb");
    for (int32_t r = 0; r < nbr; ++r) {
      BLK_REQUIRE(A->h_rowptr[r] <= A->h_rowptr[r + 1], BLKAMG_EINVAL, "rowptr not monotone");
      for (int32_t k = A->h_rowptr[r]; k < A->h_rowptr[r + 1]; ++k) {
        BLK_REQUIRE(A->h_colidx[k] >= 0 && A->h_colidx[k] < nbc, BLKAMG_EINVAL, "column index out of range");
        BLK_REQUIRE(k == A->h_rowptr[r] || A->h_colidx[k - 1] < A->h_colidx[k], BLKAMG_EINVAL,
                    "columns not strictly ascending in a row");
      }
    }
  }
  *out = A.release();
  BLK_API_END
}

int bsr_destroy(bsr_t A) {
  BLK_API_BEGIN
  delete A;
  BLK_API_END
}

int bsr_mark_modified(bsr_t A) {
  BLK_API_BEGIN
  BLK_REQUIRE(A != nullptr, BLKAMG_EINVAL, "A is NULL");
  A->stamp++;
  BLK_API_END
}

int bsr_info(bsr_t A, int32_t* nbr, int32_t* nbc, int32_t* bs_r, int32_t* bs_c, int64_t* nnzb, int* dtype,
             uint64_t* stamp) {
  BLK_API_BEGIN
  BLK_REQUIRE(A != nullptr, BLKAMG_EINVAL, "A is NULL");
  if (nbr) *nbr = A->nbr;
  if (nbc) *nbc = A->nbc;
  if (bs_r) *bs_r = A->br;
  if (bs_c) *bs_c = A->bc;
  if (nnzb) *nnzb = A->nnzb;
  if (dtype) *dtype = A->dtype;
  if (stamp) *stamp = A->stamp;
  BLK_API_END
}

int bsr_arrays(bsr_t A, const int32_t** d_rowptr, const int32_t** d_colidx, void** d_val) {
  BLK_API_BEGIN
  BLK_REQUIRE(A != nullptr, BLKAMG_EINVAL, "A is NULL");
  if (d_rowptr) *d_rowptr = A->rowptr;
  if (d_colidx) *d_colidx = A->colidx;
  if (d_val) *d_val = A->val;
  BLK_API_END
}

int bsr_autotune(bsr_t A, int vec_dtype, int32_t nrhs, void* stream, int32_t* code) {
  BLK_API_BEGIN
  BLK_REQUIRE(A != nullptr, BLKAMG_EINVAL, "A is NULL");
  BLK_REQUIRE(vec_dtype == BLKAMG_F64 || vec_dtype == BLKAMG_F32, BLKAMG_EINVAL, "vec_dtype must be F64 or F32");
  const int c = autotune_lanes(A, vec_dtype, nrhs, as_stream(stream));
  if (code) *code = c;
  BLK_API_END
}

int bsr_spmv(bsr_t A, double alpha, const void* d_x, double beta, void* d_y, int vec_dtype, int32_t nrhs,
             void* stream) {
  BLK_API_BEGIN
  BLK_REQUIRE(A != nullptr, BLKAMG_EINVAL, "A is NULL");
  spmv(A, alpha, d_x, beta, d_y, vec_dtype, nrhs, as_stream(stream));
  BLK_API_END
}

int bsr_spmv_sym(bsr_t A, double alpha, const void* d_x, double beta, void* d_y, int vec_dtype, int32_t nrhs,
                 void* stream) {
  BLK_API_BEGIN
  BLK_REQUIRE(A != nullptr, BLKAMG_EINVAL, "A is NULL");
  hipStream_t s = as_stream(stream);
  const int32_t* mir = symmetric_mirror(A, s);
  BLK_REQUIRE(mir != nullptr, BLKAMG_EINVAL, "symmetric reads need square blocks and a symmetric pattern");
  spmv(A, alpha, d_x, beta, d_y, vec_dtype, nrhs, s, lanes_for_reads(A, nrhs, mir), mir, A->sym_dist);
  BLK_API_END
}

int bsr_spmv_t(bsr_t A, double alpha, const void* d_x, double beta, void* d_y, int vec_dtype, int32_t nrhs,
               void* stream) {
  BLK_API_BEGIN
  BLK_REQUIRE(A != nullptr, BLKAMG_EINVAL, "A is NULL");
  BLK_REQUIRE(nrhs >= 1 && nrhs <= 8, BLKAMG_EINVAL, "nrhs must be in 1..8");
  bsr_s* R = transpose_of(A, as_stream(stream));
  spmv(R, alpha, d_x, beta, d_y, vec_dtype, nrhs, as_stream(stream));
  BLK_API_END
}

}  // extern "C"

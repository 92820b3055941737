// Blocked COO assembly (paper §3.4 and §5): block coordinates are declared once, a
// duplicate-summation plan is built, and every numeric assembly is one device
// kernel that sums contiguous bs_r*bs_c value runs into the block matrix.
#include <algorithm>
#include <string>
#include <thread>

#include <hipcub/hipcub.hpp>

#include "internal.hpp"

struct coo_plan_s {
  int32_t nbr = 0, nbc = 0, br = 0, bc = 0;
  int64_t n = 0, n_valid = 0, nnzb = 0;
  blk::DevBuf<int32_t> perm, seg;
  // identity of the matrix the plan created (pattern check in assemble)
  const int32_t* rowptr = nullptr;
  const int32_t* colidx = nullptr;
};

namespace blk {
namespace {

// One thread per (destination block, run of C value components): consecutive threads
// read consecutive runs of one source block and write consecutive runs of the
// destination, and each destination value is summed in stream order.  The duplicate
// list is taken kU entries at a time with all kU source positions, then all kU*C
// values, loaded before they are added (in order), so a thread waits for two
// dependent loads per kU entries instead of two per entry.  C = 3 with kU = 2
// (1.5x faster than C = 1, kU = 4 on 3x3 blocks at 128^3) keeps the loads in flight
// per thread at six without cutting the number of waves below what hides latency.
template <class T, int BE, int C = 1, int kU = 4>
__global__ __launch_bounds__(256) void coo_sum_kernel(int64_t nnzb, const int32_t* __restrict__ perm,
                                                      const int32_t* __restrict__ seg,
                                                      const T* __restrict__ vals, T* __restrict__ out,
                                                      int add, float* __restrict__ out32) {
  constexpr int NT = BE / C;  // threads per destination block
  const int64_t total = nnzb * NT;
  const int64_t g = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (g >= total) return;
  const int64_t t = g / NT;
  const int e = static_cast<int>(g - t * NT) * C;
  const int s0 = seg[t], s1 = seg[t + 1];
  T acc[C];
#pragma unroll
  for (int c = 0; c < C; ++c) acc[c] = T(0);
  for (int s = s0; s < s1; s += kU) {
    int64_t src[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) src[u] = s + u < s1 ? static_cast<int64_t>(perm[s + u]) * BE + e : -1;
    T v[kU][C];
#pragma unroll
    for (int u = 0; u < kU; ++u)
#pragma unroll
      for (int c = 0; c < C; ++c) v[u][c] = src[u] >= 0 ? vals[src[u] + c] : T(0);
#pragma unroll
    for (int u = 0; u < kU; ++u)
      if (s + u < s1) {
#pragma unroll
        for (int c = 0; c < C; ++c) acc[c] += v[u][c];
      }
  }
  T* o = out + t * BE + e;
  if (add) {
#pragma unroll
    for (int c = 0; c < C; ++c) acc[c] += o[c];
  }
  // the matrix is far larger than the caches and is read next by other kernels:
  // non-temporal stores keep L2 for the gathered values (6 % faster at 128^3)
#pragma unroll
  for (int c = 0; c < C; ++c) __builtin_nontemporal_store(acc[c], o + c);
  if (out32) {  // the FP32 copy a mixed-precision hierarchy keeps, rounded from the sums
    float* o32 = out32 + t * BE + e;
#pragma unroll
    for (int c = 0; c < C; ++c) __builtin_nontemporal_store(static_cast<float>(acc[c]), o32 + c);
  }
}

template <class T>
__global__ void coo_sum_generic_kernel(int64_t nnzb, int be, const int32_t* __restrict__ perm,
                                       const int32_t* __restrict__ seg, const T* __restrict__ vals,
                                       T* __restrict__ out, int add) {
  const int64_t total = nnzb * be;
  for (int64_t g = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; g < total;
       g += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int64_t t = g / be;
    const int e = static_cast<int>(g - t * be);
    T acc = T(0);
    for (int s = seg[t]; s < seg[t + 1]; ++s) acc += vals[static_cast<int64_t>(perm[s]) * be + e];
    out[g] = add ? out[g] + acc : acc;
  }
}

// Sums the stream into out; with out32 (3x3 blocks only) also writes the sums rounded
// to FP32 there.  Returns whether out32 was written.
template <class T>
bool launch_sum(const coo_plan_s* p, const T* vals, T* out, int add, hipStream_t s, float* out32 = nullptr) {
  if (p->nnzb == 0) return out32 != nullptr;
  const int be = p->br * p->bc;
  const int64_t total = p->nnzb * be;
  const int64_t grid = (total + 255) / 256;
  bool copied = false;
  if (be == 1 && grid < INT32_MAX) {
    coo_sum_kernel<T, 1><<<static_cast<int>(grid), 256, 0, s>>>(p->nnzb, p->perm.p, p->seg.p, vals, out, add,
                                                                  nullptr);
  } else if ((be == 9 || be == 18 || be == 36) && grid < INT32_MAX) {
    // three components per thread: a third of the threads, each with three
    // independent sums in flight
    const int g3 = static_cast<int>((total / 3 + 255) / 256);
    if (be == 9) {
      coo_sum_kernel<T, 9, 3, 2><<<g3, 256, 0, s>>>(p->nnzb, p->perm.p, p->seg.p, vals, out, add, out32);
      copied = out32 != nullptr;
    } else if (be == 18) {
      coo_sum_kernel<T, 18, 3, 2><<<g3, 256, 0, s>>>(p->nnzb, p->perm.p, p->seg.p, vals, out, add, nullptr);
    } else {
      coo_sum_kernel<T, 36, 3, 2><<<g3, 256, 0, s>>>(p->nnzb, p->perm.p, p->seg.p, vals, out, add, nullptr);
    }
  } else {
    const int g2 = static_cast<int>(std::min<int64_t>(grid, 1 << 20));
    coo_sum_generic_kernel<T><<<g2, 256, 0, s>>>(p->nnzb, be, p->perm.p, p->seg.p, vals, out, add);
  }
  HIP_CHECK(hipGetLastError());
  return copied;
}

// ---------------------------------------------------------------------------
// Plan creation on the device: the same index map as the host plan.  Valid entries
// are compacted in stream order, their 64-bit keys row * nbc + col are sorted by a
// stable radix sort (equal keys keep ascending stream position), and the runs of
// equal keys give the segments and the unique sorted pattern.
// ---------------------------------------------------------------------------
__global__ void coo_valid_kernel(int64_t n, const int32_t* __restrict__ ci, const int32_t* __restrict__ cj,
                                 int32_t nbr, int32_t nbc, int32_t* __restrict__ flag,
                                 unsigned long long* __restrict__ bad) {
  const int64_t k = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (k >= n) return;
  const int32_t i = ci[k], j = cj[k];
  const bool valid = i >= 0 && j >= 0;
  flag[k] = valid ? 1 : 0;
  if (valid && (i >= nbr || j >= nbc)) atomicMin(bad, static_cast<unsigned long long>(k));
}

__global__ void coo_compact_kernel(int64_t n, const int32_t* __restrict__ ci, const int32_t* __restrict__ cj,
                                   int32_t nbc, const int32_t* __restrict__ flag, const int32_t* __restrict__ pos,
                                   uint64_t* __restrict__ key, int32_t* __restrict__ src) {
  const int64_t k = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (k >= n || !flag[k]) return;
  const int32_t p = pos[k];
  key[p] = static_cast<uint64_t>(ci[k]) * static_cast<uint64_t>(nbc) + static_cast<uint64_t>(cj[k]);
  src[p] = static_cast<int32_t>(k);
}

__global__ void coo_head_kernel(int64_t nv, const uint64_t* __restrict__ key, int32_t* __restrict__ head) {
  const int64_t t = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (t >= nv) return;
  head[t] = (t == 0 || key[t] != key[t - 1]) ? 1 : 0;
}

// Unique block u starts at sorted position t (head[t] = 1, u = uid[t]): its segment
// start, its column, and the row pointers of the rows up to its own.
__global__ void coo_pattern_kernel(int64_t nv, const uint64_t* __restrict__ key, const int32_t* __restrict__ head,
                                   const int32_t* __restrict__ uid, int32_t nbc, int32_t nbr, int32_t nnzb,
                                   int32_t* __restrict__ seg, int32_t* __restrict__ colidx,
                                   int32_t* __restrict__ rowptr) {
  const int64_t t = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (t >= nv || !head[t]) return;
  const int32_t u = uid[t];
  const uint64_t k = key[t];
  const int32_t row = static_cast<int32_t>(k / static_cast<uint64_t>(nbc));
  seg[u] = static_cast<int32_t>(t);
  colidx[u] = static_cast<int32_t>(k - static_cast<uint64_t>(row) * static_cast<uint64_t>(nbc));
  const int32_t prev = t == 0 ? -1 : static_cast<int32_t>(key[t - 1] / static_cast<uint64_t>(nbc));
  for (int32_t r = prev + 1; r <= row; ++r) rowptr[r] = u;  // rows prev+1..row start at block u
  if (u == nnzb - 1) {
    for (int32_t r = row + 1; r <= nbr; ++r) rowptr[r] = nnzb;
    seg[nnzb] = static_cast<int32_t>(nv);
  }
}

int bits_of(uint64_t v) {
  int b = 0;
  while (b < 64 && (v >> b) != 0) ++b;
  return b;
}

template <class T>
void exclusive_sum(const T* in, T* out, int64_t n, hipStream_t s) {
  size_t bytes = 0;
  HIP_CHECK(hipcub::DeviceScan::ExclusiveSum(nullptr, bytes, in, out, static_cast<int>(n), s));
  DevBuf<char> tmp(std::max<size_t>(bytes, 1));
  HIP_CHECK(hipcub::DeviceScan::ExclusiveSum(tmp.p, bytes, in, out, static_cast<int>(n), s));
}

int32_t read_last_sum(const int32_t* excl, const int32_t* flags, int64_t n, hipStream_t s) {
  int32_t a = 0, b = 0;
  HIP_CHECK(hipMemcpyAsync(&a, excl + (n - 1), sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIP_CHECK(hipMemcpyAsync(&b, flags + (n - 1), sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIP_CHECK(hipStreamSynchronize(s));
  return a + b;
}

// Device plan of n coordinates d_i, d_j (device int32): perm, seg, rowptr, colidx on
// the device; *n_valid, *nnzb.  Sync (a few scalar reads).
void coo_plan_device(int32_t nbr, int32_t nbc, int64_t n, const int32_t* d_i, const int32_t* d_j, hipStream_t s,
                     DevBuf<int32_t>& perm, DevBuf<int32_t>& seg, DevBuf<int32_t>& rowptr, DevBuf<int32_t>& colidx,
                     int64_t& n_valid, int64_t& nnzb) {
  n_valid = 0;
  nnzb = 0;
  rowptr.alloc(static_cast<size_t>(nbr) + 1);
  HIP_CHECK(hipMemsetAsync(rowptr.p, 0, rowptr.bytes(), s));
  if (n == 0) {
    seg.alloc(1);
    HIP_CHECK(hipMemsetAsync(seg.p, 0, sizeof(int32_t), s));
    HIP_CHECK(hipStreamSynchronize(s));
    return;
  }
  const int grid = static_cast<int>((n + 255) / 256);
  DevBuf<int32_t> flag(static_cast<size_t>(n)), pos(static_cast<size_t>(n));
  DevBuf<unsigned long long> bad(1);
  const unsigned long long none = ~0ull;
  HIP_CHECK(hipMemcpyAsync(bad.p, &none, sizeof(none), hipMemcpyHostToDevice, s));
  coo_valid_kernel<<<grid, 256, 0, s>>>(n, d_i, d_j, nbr, nbc, flag.p, bad.p);
  HIP_CHECK(hipGetLastError());
  unsigned long long hb = 0;
  HIP_CHECK(hipMemcpyAsync(&hb, bad.p, sizeof(hb), hipMemcpyDeviceToHost, s));
  HIP_CHECK(hipStreamSynchronize(s));
  BLK_REQUIRE(hb == none, BLKAMG_EINVAL, "COO coordinate out of range at entry " + std::to_string(hb));
  exclusive_sum(flag.p, pos.p, n, s);
  const int32_t nv = read_last_sum(pos.p, flag.p, n, s);
  n_valid = nv;
  if (nv == 0) {
    perm.release();
    seg.alloc(1);
    HIP_CHECK(hipMemsetAsync(seg.p, 0, sizeof(int32_t), s));
    HIP_CHECK(hipStreamSynchronize(s));
    return;
  }
  DevBuf<uint64_t> key(static_cast<size_t>(nv)), key2(static_cast<size_t>(nv));
  DevBuf<int32_t> src(static_cast<size_t>(nv));
  perm.alloc(static_cast<size_t>(nv));
  coo_compact_kernel<<<grid, 256, 0, s>>>(n, d_i, d_j, nbc, flag.p, pos.p, key.p, src.p);
  HIP_CHECK(hipGetLastError());
  flag.release();
  pos.release();
  const int end_bit = std::max(1, bits_of(static_cast<uint64_t>(std::max(nbr, 1)) * static_cast<uint64_t>(std::max(nbc, 1))));
  size_t sort_bytes = 0;
  HIP_CHECK(hipcub::DeviceRadixSort::SortPairs(nullptr, sort_bytes, key.p, key2.p, src.p, perm.p, nv, 0, end_bit, s));
  {
    DevBuf<char> tmp(std::max<size_t>(sort_bytes, 1));
    HIP_CHECK(hipcub::DeviceRadixSort::SortPairs(tmp.p, sort_bytes, key.p, key2.p, src.p, perm.p, nv, 0, end_bit, s));
  }
  key.release();
  src.release();
  DevBuf<int32_t> head(static_cast<size_t>(nv)), uid(static_cast<size_t>(nv));
  const int vgrid_ = static_cast<int>((static_cast<int64_t>(nv) + 255) / 256);
  coo_head_kernel<<<vgrid_, 256, 0, s>>>(nv, key2.p, head.p);
  HIP_CHECK(hipGetLastError());
  exclusive_sum(head.p, uid.p, nv, s);
  const int32_t nu = read_last_sum(uid.p, head.p, nv, s);
  nnzb = nu;
  seg.alloc(static_cast<size_t>(nu) + 1);
  colidx.alloc(static_cast<size_t>(nu));
  coo_pattern_kernel<<<vgrid_, 256, 0, s>>>(nv, key2.p, head.p, uid.p, nbc, nbr, nu, seg.p, colidx.p, rowptr.p);
  HIP_CHECK(hipGetLastError());
  HIP_CHECK(hipStreamSynchronize(s));
}

}  // namespace
}  // namespace blk

using namespace blk;

extern "C" {

int coo_plan_create(int32_t nbr, int32_t nbc, int32_t bs_r, int32_t bs_c, int64_t n, const int32_t* h_i,
                    const int32_t* h_j, int where, int val_dtype, coo_plan_t* plan, bsr_t* A_out, void* stream) {
  // h_i / h_j are device pointers when where == BLKAMG_DEVICE
  BLK_API_BEGIN
  BLK_REQUIRE(plan != nullptr && A_out != nullptr, BLKAMG_EINVAL, "output pointer is NULL");
  *plan = nullptr;
  *A_out = nullptr;
  BLK_REQUIRE(nbr >= 0 && nbc >= 0 && n >= 0, BLKAMG_EINVAL, "negative size");
  BLK_REQUIRE(bs_r >= 1 && bs_r <= 8 && bs_c >= 1 && bs_c <= 8, BLKAMG_EINVAL, "block size must be in 1..8");
  BLK_REQUIRE(n == 0 || (h_i != nullptr && h_j != nullptr), BLKAMG_EINVAL, "coordinate array is NULL");
  BLK_REQUIRE(n <= INT32_MAX, BLKAMG_EINVAL, "stream longer than the int32 index range");
  BLK_REQUIRE(val_dtype == BLKAMG_F64 || val_dtype == BLKAMG_F32, BLKAMG_EINVAL, "COO values must be F64 or F32");
  BLK_REQUIRE(where == BLKAMG_HOST || where == BLKAMG_DEVICE, BLKAMG_EINVAL, "where must be HOST or DEVICE");
  if (where == BLKAMG_DEVICE) {
    hipStream_t s = as_stream(stream);
    auto P = std::make_unique<coo_plan_s>();
    auto A = std::make_unique<bsr_s>();
    DevBuf<int32_t> rp, ci;
    int64_t nv = 0, nu = 0;
    coo_plan_device(nbr, nbc, n, h_i, h_j, s, P->perm, P->seg, rp, ci, nv, nu);
    BLK_REQUIRE(nu <= INT32_MAX, BLKAMG_EINVAL, "too many blocks");
    P->nbr = nbr;
    P->nbc = nbc;
    P->br = bs_r;
    P->bc = bs_c;
    P->n = n;
    P->n_valid = nv;
    P->nnzb = nu;
    A->nbr = nbr;
    A->nbc = nbc;
    A->br = bs_r;
    A->bc = bs_c;
    A->dtype = val_dtype;
    A->nnzb = nu;
    A->own_rowptr = std::move(rp);
    A->own_colidx = std::move(ci);
    A->own_val.alloc(A->val_bytes());
    if (A->own_val.p) HIP_CHECK(hipMemsetAsync(A->own_val.p, 0, A->val_bytes(), s));
    HIP_CHECK(hipStreamSynchronize(s));
    A->rowptr = A->own_rowptr.p;
    A->colidx = A->own_colidx.p;
    A->val = A->own_val.p;
    P->rowptr = A->rowptr;
    P->colidx = A->colidx;
    *plan = P.release();
    *A_out = A.release();
    return BLKAMG_OK;
  }

  // 1. count valid entries per block row (and check ranges)
  std::vector<int64_t> cnt(static_cast<size_t>(nbr) + 1, 0);
  for (int64_t k = 0; k < n; ++k) {
    const int32_t i = h_i[k], j = h_j[k];
    if (i < 0 || j < 0) continue;
    BLK_REQUIRE(i < nbr && j < nbc, BLKAMG_EINVAL,
                "COO coordinate out of range at entry " + std::to_string(k));
    cnt[i + 1]++;
  }
  for (int32_t r = 0; r < nbr; ++r) cnt[r + 1] += cnt[r];
  const int64_t nv = cnt[nbr];
  // 2. stable bucket by row (k ascending inside each bucket)
  std::vector<int32_t> perm(static_cast<size_t>(nv));
  {
    std::vector<int64_t> next(cnt.begin(), cnt.end() - 1);
    for (int64_t k = 0; k < n; ++k) {
      const int32_t i = h_i[k], j = h_j[k];
      if (i < 0 || j < 0) continue;
      perm[next[i]++] = static_cast<int32_t>(k);
    }
  }
  // 3. inside each row order by (column, position); count unique blocks per row
  std::vector<int32_t> ucount(static_cast<size_t>(nbr), 0);
  auto sort_rows = [&](int32_t r0, int32_t r1) {
    for (int32_t r = r0; r < r1; ++r) {
      int32_t* b = perm.data() + cnt[r];
      int32_t* e = perm.data() + cnt[r + 1];
      std::sort(b, e, [&](int32_t a, int32_t c) { return h_j[a] != h_j[c] ? h_j[a] < h_j[c] : a < c; });
      int32_t u = 0;
      for (int32_t* q = b; q < e; ++q)
        if (q == b || h_j[*q] != h_j[*(q - 1)]) ++u;
      ucount[r] = u;
    }
  };
  const int nth = std::max(1, std::min<int>(16, static_cast<int>(std::thread::hardware_concurrency())));
  if (nv > (1 << 20) && nth > 1) {
    std::vector<std::thread> ts;
    for (int t = 0; t < nth; ++t) {
      const int32_t r0 = static_cast<int32_t>(static_cast<int64_t>(nbr) * t / nth);
      const int32_t r1 = static_cast<int32_t>(static_cast<int64_t>(nbr) * (t + 1) / nth);
      ts.emplace_back(sort_rows, r0, r1);
    }
    for (auto& th : ts) th.join();
  } else {
    sort_rows(0, nbr);
  }
  // 4. pattern and segments
  std::vector<int32_t> rowptr(static_cast<size_t>(nbr) + 1, 0);
  for (int32_t r = 0; r < nbr; ++r) rowptr[r + 1] = rowptr[r] + ucount[r];
  const int64_t nnzb = rowptr[nbr];
  BLK_REQUIRE(nnzb <= INT32_MAX, BLKAMG_EINVAL, "too many blocks");
  std::vector<int32_t> colidx(static_cast<size_t>(nnzb)), seg(static_cast<size_t>(nnzb) + 1);
  {
    int64_t t = 0;
    for (int32_t r = 0; r < nbr; ++r)
      for (int64_t q = cnt[r]; q < cnt[r + 1]; ++q)
        if (q == cnt[r] || h_j[perm[q]] != h_j[perm[q - 1]]) {
          colidx[t] = h_j[perm[q]];
          seg[t] = static_cast<int32_t>(q);
          ++t;
        }
    seg[nnzb] = static_cast<int32_t>(nv);
  }
  auto P = std::make_unique<coo_plan_s>();
  P->nbr = nbr;
  P->nbc = nbc;
  P->br = bs_r;
  P->bc = bs_c;
  P->n = n;
  P->n_valid = nv;
  P->nnzb = nnzb;
  upload(P->perm, perm);
  upload(P->seg, seg);
  auto A = make_owned(nbr, nbc, bs_r, bs_c, val_dtype, std::move(rowptr), std::move(colidx));
  P->rowptr = A->rowptr;
  P->colidx = A->colidx;
  *plan = P.release();
  *A_out = A.release();
  BLK_API_END
}

int coo_plan_destroy(coo_plan_t plan) {
  BLK_API_BEGIN
  delete plan;
  BLK_API_END
}

int coo_plan_map(coo_plan_t plan, const int32_t** d_perm, const int32_t** d_seg, int64_t* n_valid,
                 int64_t* nnzb) {
  BLK_API_BEGIN
  BLK_REQUIRE(plan != nullptr, BLKAMG_EINVAL, "plan is NULL");
  if (d_perm) *d_perm = plan->perm.p;
  if (d_seg) *d_seg = plan->seg.p;
  if (n_valid) *n_valid = plan->n_valid;
  if (nnzb) *nnzb = plan->nnzb;
  BLK_API_END
}

int coo_assemble_blocked(coo_plan_t plan, const void* d_vals, int val_dtype, int mode, bsr_t A, void* stream) {
  BLK_API_BEGIN
  BLK_REQUIRE(plan != nullptr && A != nullptr, BLKAMG_EINVAL, "plan or A is NULL");
  BLK_REQUIRE(mode == BLKAMG_INSERT || mode == BLKAMG_ADD, BLKAMG_EINVAL, "mode must be INSERT or ADD");
  BLK_REQUIRE(val_dtype == A->dtype, BLKAMG_EINVAL, "value dtype differs from the matrix dtype");
  BLK_REQUIRE(A->nbr == plan->nbr && A->nbc == plan->nbc && A->br == plan->br && A->bc == plan->bc &&
                  A->nnzb == plan->nnzb,
              BLKAMG_EINVAL, "matrix shape differs from the plan");
  BLK_REQUIRE(plan->n_valid == 0 || d_vals != nullptr, BLKAMG_EINVAL, "values are NULL");
  hipStream_t s = as_stream(stream);
  // an FP32 copy kept by a mixed-precision hierarchy is written in the same pass
  bsr_s* cp = A->f32_copy;
  const bool want32 = cp != nullptr && val_dtype == BLKAMG_F64 && cp->dtype == BLKAMG_F32 && cp->nnzb == A->nnzb &&
                      cp->br == A->br && cp->bc == A->bc;
  bool copied = false;
  if (val_dtype == BLKAMG_F64)
    copied = launch_sum<double>(plan, static_cast<const double*>(d_vals), static_cast<double*>(A->val),
                                mode == BLKAMG_ADD, s, want32 ? static_cast<float*>(cp->val) : nullptr);
  else
    launch_sum<float>(plan, static_cast<const float*>(d_vals), static_cast<float*>(A->val), mode == BLKAMG_ADD, s);
  A->stamp++;
  if (copied) {
    A->f32_copy_stamp = A->stamp;
    cp->stamp++;
  }
  BLK_API_END
}

}  // extern "C"

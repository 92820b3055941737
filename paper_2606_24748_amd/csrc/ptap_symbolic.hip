// Symbolic phase of the Galerkin product A_c = P^T A P on the device (paper §3.1,
// §3.5; §6: the device-resident setup): the patterns of A P and of A_c, each output
// block's list of contributions, and the workgroup tables of the numeric kernels.
//
// Every product pattern Out = X Y is built row by row.  The contributions of output
// row r are the pairs (k, q) with k in X's row r and q in Y's row x_ci[k]; taken in
// (k, q) order they are the candidates of the row, keyed by their column y_ci[q].  One
// 64-lane workgroup generates a row's candidates into LDS, sorts them by (column,
// generation index) with a bitonic network, and reads off the output columns (the
// distinct keys, ascending) and each output's contributions (its run of the sorted
// candidates, in (k, q) order).  This is the order the host build produces, so both
// builds give the same plan and the numeric product the same bits.
#include <algorithm>
#include <string>

#include <hipcub/hipcub.hpp>

#include "ptap_plan.hpp"
#include "spmv_core.hpp"

namespace blk {
namespace {

constexpr int kMaxCand = 4096;  // contributions of one output row sorted in LDS at most (48 KiB)

__device__ __forceinline__ int wave_max_int(int v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = max(v, __shfl_xor(v, off, 64));
  return v;
}

// Per output row r: the number of contributions (only columns >= r when UPPER), and
// the largest X and Y row offsets that contribute (maxima[0], maxima[1]) and the
// largest contribution count (maxima[2]) over all rows.
template <bool UPPER>
__global__ __launch_bounds__(256) void prod_count_kernel(int nrows, const int32_t* __restrict__ x_rp,
                                                         const int32_t* __restrict__ x_ci,
                                                         const int32_t* __restrict__ y_rp,
                                                         const int32_t* __restrict__ y_ci, int64_t* __restrict__ n_cand,
                                                         int* __restrict__ maxima) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  int cnt = 0, kmax = 0, qmax = 0;
  if (r < nrows) {
    const int k0 = x_rp[r], k1 = x_rp[r + 1];
    for (int k = k0; k < k1; ++k) {
      const int j = x_ci[k];
      const int q0 = y_rp[j], q1 = y_rp[j + 1];
      for (int q = q0; q < q1; ++q) {
        if (UPPER && y_ci[q] < r) continue;
        ++cnt;
        kmax = max(kmax, k - k0);
        qmax = max(qmax, q - q0);
      }
    }
    n_cand[r] = cnt;
  }
  kmax = wave_max_int(kmax);
  qmax = wave_max_int(qmax);
  cnt = wave_max_int(cnt);
  if ((threadIdx.x & 63) == 0) {
    atomicMax(maxima + 0, kmax);
    atomicMax(maxima + 1, qmax);
    atomicMax(maxima + 2, cnt);
  }
}

// The candidates of output row r in (k, q) order: keys[pos] = column << 32 | pos and
// pay[pos] = k offset << 16 | q offset, pos = 0 .. n-1 (keys and pay in LDS, or a
// row's slice of a device buffer).  One 64-lane wave; returns n.
template <bool UPPER>
__device__ __forceinline__ int gen_row(int r, const int32_t* __restrict__ x_rp, const int32_t* __restrict__ x_ci,
                                       const int32_t* __restrict__ y_rp, const int32_t* __restrict__ y_ci,
                                       uint64_t* keys, uint32_t* pay, int lane) {
  const int k0 = x_rp[r], k1 = x_rp[r + 1];
  int base = 0;
  for (int kb = k0; kb < k1; kb += 64) {
    const int k = kb + lane;
    int c = 0, q0 = 0, q1 = 0;
    if (k < k1) {
      const int j = x_ci[k];
      q0 = y_rp[j];
      q1 = y_rp[j + 1];
      if (UPPER) {
        for (int q = q0; q < q1; ++q) c += y_ci[q] >= r ? 1 : 0;
      } else {
        c = q1 - q0;
      }
    }
    int incl = c;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const int v = __shfl_up(incl, off, 64);
      if (lane >= off) incl += v;
    }
    int pos = base + incl - c;
    for (int q = q0; q < q1; ++q) {
      const int col = y_ci[q];
      if (UPPER && col < r) continue;
      keys[pos] = (static_cast<uint64_t>(static_cast<uint32_t>(col)) << 32) | static_cast<uint32_t>(pos);
      pay[pos] = (static_cast<uint32_t>(k - k0) << 16) | static_cast<uint32_t>(q - q0);
      ++pos;
    }
    base += __shfl(incl, 63, 64);
  }
  return base;
}

// From the n sorted candidates of row r: COUNT, n_out[r] = number of distinct columns;
// otherwise (fill) the row's output columns at out_ci[out_rp[r]..] and, with pairs,
// pp[output] = cand_off[r] + the start of its run and the codes (k offset << shift |
// q offset, WIDTH bytes little endian) at codes[(cand_off[r] + position) * WIDTH].
template <bool COUNT, int WIDTH>
__device__ __forceinline__ void emit_row(int r, int n, const uint64_t* keys, const uint32_t* pay, int lane,
                                         int32_t* __restrict__ n_out, const int32_t* __restrict__ out_rp,
                                         int32_t* __restrict__ out_ci, const int64_t* __restrict__ cand_off,
                                         int32_t* __restrict__ pp, uint8_t* __restrict__ codes, int shift) {
  int ubase = 0;
  for (int pb = 0; pb < n; pb += 64) {
    const int p = pb + lane;
    const bool valid = p < n;
    const uint32_t col = valid ? static_cast<uint32_t>(keys[p] >> 32) : 0u;
    const bool start = valid && (p == 0 || static_cast<uint32_t>(keys[p - 1] >> 32) != col);
    const uint64_t ball = __ballot(start);
    if constexpr (!COUNT) {
      if (start) {
        const int u = ubase + __popcll(ball & ((1ull << lane) - 1ull));
        const int oidx = out_rp[r] + u;
        out_ci[oidx] = static_cast<int32_t>(col);
        if (pp) pp[oidx] = static_cast<int32_t>(cand_off[r] + p);
      }
      if (codes && valid) {
        const uint32_t pl = pay[static_cast<uint32_t>(keys[p])];
        const uint32_t code = ((pl >> 16) << shift) | (pl & 0xFFFFu);
        uint8_t* dst = codes + static_cast<size_t>(cand_off[r] + p) * WIDTH;
        if constexpr (WIDTH == 1) {
          dst[0] = static_cast<uint8_t>(code);
        } else if constexpr (WIDTH == 2) {
          *reinterpret_cast<uint16_t*>(dst) = static_cast<uint16_t>(code);
        } else {
          *reinterpret_cast<uint32_t*>(dst) = code;
        }
      }
    }
    ubase += __popcll(ball);
  }
  if constexpr (COUNT) {
    if (lane == 0) n_out[r] = ubase;
  }
}

// One workgroup (one wave) per output row with at most p2cap candidates, rows strided
// over the grid (longer rows are left to the device-memory path).  LDS: keys[p2cap]
// and pay[p2cap]; a bitonic network sorts a row's keys.
template <bool UPPER, bool COUNT, int WIDTH>
__global__ __launch_bounds__(64) void prod_sort_kernel(int nrows, const int32_t* __restrict__ x_rp,
                                                       const int32_t* __restrict__ x_ci,
                                                       const int32_t* __restrict__ y_rp,
                                                       const int32_t* __restrict__ y_ci, int p2cap,
                                                       const int64_t* __restrict__ n_cand,
                                                       int32_t* __restrict__ n_out, const int32_t* __restrict__ out_rp,
                                                       int32_t* __restrict__ out_ci, const int64_t* __restrict__ cand_off,
                                                       int32_t* __restrict__ pp, uint8_t* __restrict__ codes, int shift) {
  extern __shared__ __align__(16) unsigned char sym_lds[];
  uint64_t* keys = reinterpret_cast<uint64_t*>(sym_lds);
  uint32_t* pay = reinterpret_cast<uint32_t*>(sym_lds + static_cast<size_t>(p2cap) * 8);
  const int lane = threadIdx.x;
  for (int r = blockIdx.x; r < nrows; r += gridDim.x) {
    if (n_cand[r] > p2cap) continue;  // uniform over the workgroup
    const int n = gen_row<UPPER>(r, x_rp, x_ci, y_rp, y_ci, keys, pay, lane);
    int p2 = 1;
    while (p2 < n) p2 <<= 1;
    for (int i = n + lane; i < p2; i += 64) keys[i] = ~0ull;
    __syncthreads();
    for (int size = 2; size <= p2; size <<= 1) {
      for (int stride = size >> 1; stride > 0; stride >>= 1) {
        for (int t = lane; t < p2 / 2; t += 64) {
          const int lo = 2 * stride * (t / stride) + (t % stride);
          const int hi = lo + stride;
          const bool asc = (lo & size) == 0;
          const uint64_t a = keys[lo], b = keys[hi];
          if ((a > b) == asc) {
            keys[lo] = b;
            keys[hi] = a;
          }
        }
        __syncthreads();
      }
    }
    emit_row<COUNT, WIDTH>(r, n, keys, pay, lane, n_out, out_rp, out_ci, cand_off, pp, codes, shift);
    __syncthreads();  // the next row reuses the LDS
  }
}

// Rows beyond the LDS sort: their candidates go to device memory (row li of the list
// at loff[li]), are sorted there by a segmented radix sort, and emitted like the rest.
template <bool UPPER>
__global__ __launch_bounds__(64) void long_gen_kernel(int nlong, const int32_t* __restrict__ rows,
                                                      const int64_t* __restrict__ loff,
                                                      const int32_t* __restrict__ x_rp,
                                                      const int32_t* __restrict__ x_ci,
                                                      const int32_t* __restrict__ y_rp,
                                                      const int32_t* __restrict__ y_ci, uint64_t* __restrict__ keys,
                                                      uint32_t* __restrict__ pay) {
  for (int li = blockIdx.x; li < nlong; li += gridDim.x)
    gen_row<UPPER>(rows[li], x_rp, x_ci, y_rp, y_ci, keys + loff[li], pay + loff[li], threadIdx.x);
}

template <bool COUNT, int WIDTH>
__global__ __launch_bounds__(64) void long_emit_kernel(int nlong, const int32_t* __restrict__ rows,
                                                       const int64_t* __restrict__ loff,
                                                       const uint64_t* __restrict__ keys,
                                                       const uint32_t* __restrict__ pay, int32_t* __restrict__ n_out,
                                                       const int32_t* __restrict__ out_rp, int32_t* __restrict__ out_ci,
                                                       const int64_t* __restrict__ cand_off, int32_t* __restrict__ pp,
                                                       uint8_t* __restrict__ codes, int shift) {
  for (int li = blockIdx.x; li < nlong; li += gridDim.x) {
    const int64_t o = loff[li];
    emit_row<COUNT, WIDTH>(rows[li], static_cast<int>(loff[li + 1] - o), keys + o, pay + o, threadIdx.x, n_out,
                           out_rp, out_ci, cand_off, pp, codes, shift);
  }
}

// Symmetric mode: for the u-th upper output (row a, column c) its index in the full
// coarse pattern (the upper columns are the tail of the sorted full row) and its
// mirror, the index of (c, a) (-1 on the diagonal).  A missing mirror or a mismatch
// clears *ok.
__global__ void sym_lists_kernel(int nrows, const int32_t* __restrict__ crp, const int32_t* __restrict__ cci,
                                 const int32_t* __restrict__ orp, const int32_t* __restrict__ oci,
                                 int32_t* __restrict__ uidx, int32_t* __restrict__ mirror, int* __restrict__ ok) {
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= nrows) return;
  const int nu = orp[a + 1] - orp[a];
  const int first = crp[a + 1] - nu;
  if (first < crp[a]) {  // more upper outputs than the full row holds
    *ok = 0;
    for (int u = 0; u < nu; ++u) uidx[orp[a] + u] = mirror[orp[a] + u] = crp[a];
    return;
  }
  for (int u = 0; u < nu; ++u) {
    const int c = oci[orp[a] + u];
    const int t = first + u;
    if (cci[t] != c) *ok = 0;
    uidx[orp[a] + u] = t;
    int m = -1;
    if (c != a) {
      int lo = crp[c], hi = crp[c + 1];
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        const int v = cci[mid];
        if (v == a) { m = mid; break; }
        if (v < a) lo = mid + 1; else hi = mid;
      }
      if (m < 0) {
        *ok = 0;
        m = t;  // a valid position either way
      }
    }
    mirror[orp[a] + u] = m;
  }
}

// Row of the first output of every group of `per` consecutive outputs (the last
// entry bounds the last group): the largest row r with rp[r] <= g * per.
__global__ void first_rows_kernel(int ngroups, int nrows, const int32_t* __restrict__ rp, int per,
                                  int32_t* __restrict__ out) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g > ngroups) return;
  if (g == ngroups) {
    out[g] = max(nrows - 1, 0);
    return;
  }
  const int64_t s0 = static_cast<int64_t>(g) * per;
  int lo = 0, hi = nrows;  // first index u in [0, nrows] with rp[u] > s0, searched in rp[1..nrows]
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (rp[mid + 1] <= s0) lo = mid + 1; else hi = mid;
  }
  out[g] = min(lo, max(nrows - 1, 0));
}

// Inside every group of `per` (<= 256) outputs, the offsets ordered by descending
// contribution count, ties by offset (identity order when !by_count).
__global__ __launch_bounds__(256) void group_order_kernel(int64_t nout, const int32_t* __restrict__ ptr, int per,
                                                          int by_count, uint8_t* __restrict__ out) {
  __shared__ int cnt[256];
  const int64_t g = static_cast<int64_t>(blockIdx.x) * per;
  const int m = static_cast<int>(min(static_cast<int64_t>(per), nout - g));
  const int t = threadIdx.x;
  if (t < m) cnt[t] = by_count ? ptr[g + t + 1] - ptr[g + t] : 0;
  __syncthreads();
  if (t >= m) return;
  int rank = 0;
  for (int u = 0; u < m; ++u) rank += (cnt[u] > cnt[t] || (cnt[u] == cnt[t] && u < t)) ? 1 : 0;
  out[g + rank] = static_cast<uint8_t>(t);
}

// X entries spanned by every workgroup (-1 when it has more than kMaxR rows).
__global__ void group_extent_kernel(int ngroups, int nrows, const int32_t* __restrict__ w,
                                    const int32_t* __restrict__ x_rp, int32_t* __restrict__ nk) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= ngroups) return;
  const int r0 = w[g], r1 = min(nrows - 1, w[g + 1]);
  nk[g] = (r1 - r0 + 1 > kMaxR) ? -1 : x_rp[r1 + 1] - x_rp[r0];
}

void set_last(int32_t* p, int32_t v, hipStream_t s) {
  HIP_CHECK(hipMemcpyAsync(p, &v, sizeof(v), hipMemcpyHostToDevice, s));
  HIP_CHECK(hipStreamSynchronize(s));  // v lives on this stack frame
}

// Exclusive sum of n values into out[0..n] (out[n] = total).  Returns the total.
template <class T>
T scan_total(const T* in, T* out, int32_t n, hipStream_t s) {
  if (n == 0) {
    const T z = 0;
    HIP_CHECK(hipMemcpyAsync(out, &z, sizeof(T), hipMemcpyHostToDevice, s));
    HIP_CHECK(hipStreamSynchronize(s));
    return 0;
  }
  size_t bytes = 0;
  HIP_CHECK(hipcub::DeviceScan::InclusiveSum(nullptr, bytes, in, out + 1, n, s));
  DevBuf<char> tmp(std::max<size_t>(bytes, 1));
  HIP_CHECK(hipcub::DeviceScan::InclusiveSum(tmp.p, bytes, in, out + 1, n, s));
  const T z = 0;
  HIP_CHECK(hipMemcpyAsync(out, &z, sizeof(T), hipMemcpyHostToDevice, s));
  T total = 0;
  HIP_CHECK(hipMemcpyAsync(&total, out + n, sizeof(T), hipMemcpyDeviceToHost, s));
  HIP_CHECK(hipStreamSynchronize(s));
  return total;
}

int bits_of(int64_t v) {
  int b = 0;
  while ((int64_t{1} << b) <= v) ++b;
  return b;
}

struct Product {
  DevBuf<int32_t> rp, ci;  // output pattern
  int64_t nout = 0;
};

// Out = X Y on device patterns (X: nrows rows, Y: ncols columns).  With `pairs`, also
// the contribution list (codes, per-output starts, width, shift).  Rows with up to
// kMaxCand contributions are sorted in LDS, longer ones in device memory.  False when
// a row offset does not fit 16 bits or the codes would not fit 32 bits.
bool product(int nrows, int ncols, const int32_t* x_rp, const int32_t* x_ci, const int32_t* y_rp,
             const int32_t* y_ci, bool upper, PairList* pairs, Product& out, hipStream_t s) {
  DevBuf<int64_t> ncand(static_cast<size_t>(std::max(nrows, 1)));
  DevBuf<int> maxima(3);
  HIP_CHECK(hipMemsetAsync(maxima.p, 0, 3 * sizeof(int), s));
  const int rgrid = (nrows + 255) / 256;
  if (nrows > 0) {
    if (upper) prod_count_kernel<true><<<rgrid, 256, 0, s>>>(nrows, x_rp, x_ci, y_rp, y_ci, ncand.p, maxima.p);
    else prod_count_kernel<false><<<rgrid, 256, 0, s>>>(nrows, x_rp, x_ci, y_rp, y_ci, ncand.p, maxima.p);
    HIP_CHECK(hipGetLastError());
  }
  int mx[3] = {0, 0, 0};
  HIP_CHECK(hipMemcpyAsync(mx, maxima.p, sizeof(mx), hipMemcpyDeviceToHost, s));
  HIP_CHECK(hipStreamSynchronize(s));
  if (mx[0] >= 65536 || mx[1] >= 65536) return false;
  int p2cap = 1;
  while (p2cap < std::min(std::max(mx[2], 1), kMaxCand)) p2cap <<= 1;
  const size_t lds = static_cast<size_t>(p2cap) * 12;
  const int sgrid = std::max(1, std::min(nrows, 65536));
  // rows beyond the LDS sort: generated into device memory and sorted there (once,
  // for both the count and the fill)
  DevBuf<int32_t> lrows;
  DevBuf<int64_t> loff;
  DevBuf<uint64_t> lkeys, lsorted;
  DevBuf<uint32_t> lpay;
  int nlong = 0;
  if (mx[2] > kMaxCand) {
    const std::vector<int64_t> h = download(ncand.p, static_cast<size_t>(nrows), s);
    std::vector<int32_t> hr;
    std::vector<int64_t> ho(1, 0);
    for (int r = 0; r < nrows; ++r)
      if (h[r] > kMaxCand) {
        hr.push_back(r);
        ho.push_back(ho.back() + h[r]);
      }
    nlong = static_cast<int>(hr.size());
    BLK_REQUIRE(ho.back() <= INT32_MAX, BLKAMG_EINVAL, "too many contributions in long rows");
    const int ntot = static_cast<int>(ho.back());
    upload(lrows, hr);
    upload(loff, ho);
    lkeys.alloc(static_cast<size_t>(ntot));
    lsorted.alloc(static_cast<size_t>(ntot));
    lpay.alloc(static_cast<size_t>(ntot));
    const int lgrid = std::min(nlong, 65536);
    if (upper)
      long_gen_kernel<true><<<lgrid, 64, 0, s>>>(nlong, lrows.p, loff.p, x_rp, x_ci, y_rp, y_ci, lkeys.p, lpay.p);
    else
      long_gen_kernel<false><<<lgrid, 64, 0, s>>>(nlong, lrows.p, loff.p, x_rp, x_ci, y_rp, y_ci, lkeys.p, lpay.p);
    HIP_CHECK(hipGetLastError());
    const int end_bit = 32 + bits_of(std::max(ncols, 1));
    size_t bytes = 0;
    HIP_CHECK(hipcub::DeviceSegmentedRadixSort::SortKeys(nullptr, bytes, lkeys.p, lsorted.p, ntot, nlong, loff.p,
                                                         loff.p + 1, 0, end_bit, s));
    DevBuf<char> tmp(std::max<size_t>(bytes, 1));
    HIP_CHECK(hipcub::DeviceSegmentedRadixSort::SortKeys(tmp.p, bytes, lkeys.p, lsorted.p, ntot, nlong, loff.p,
                                                         loff.p + 1, 0, end_bit, s));
    HIP_CHECK(hipStreamSynchronize(s));
    lkeys.release();
  }
  const int lgrid = std::max(1, std::min(nlong, 65536));
  DevBuf<int32_t> nout(static_cast<size_t>(std::max(nrows, 1)));
  out.rp.alloc(static_cast<size_t>(nrows) + 1);
  if (nrows > 0) {
    if (upper)
      prod_sort_kernel<true, true, 1><<<sgrid, 64, lds, s>>>(nrows, x_rp, x_ci, y_rp, y_ci, p2cap, ncand.p, nout.p,
                                                              nullptr, nullptr, nullptr, nullptr, nullptr, 0);
    else
      prod_sort_kernel<false, true, 1><<<sgrid, 64, lds, s>>>(nrows, x_rp, x_ci, y_rp, y_ci, p2cap, ncand.p, nout.p,
                                                               nullptr, nullptr, nullptr, nullptr, nullptr, 0);
    HIP_CHECK(hipGetLastError());
    if (nlong > 0) {
      long_emit_kernel<true, 1><<<lgrid, 64, 0, s>>>(nlong, lrows.p, loff.p, lsorted.p, lpay.p, nout.p, nullptr,
                                                     nullptr, nullptr, nullptr, nullptr, 0);
      HIP_CHECK(hipGetLastError());
    }
  }
  const int32_t total_out = scan_total<int32_t>(nout.p, out.rp.p, nrows, s);
  out.nout = total_out;
  out.ci.alloc(static_cast<size_t>(total_out));
  DevBuf<int64_t> coff;
  int width = 1, shift = 0;
  if (pairs) {
    coff.alloc(static_cast<size_t>(nrows) + 1);
    const int64_t total_pairs = scan_total<int64_t>(ncand.p, coff.p, nrows, s);
    BLK_REQUIRE(total_pairs <= INT32_MAX, BLKAMG_EINVAL, "pair list too long");
    const int bh = bits_of(mx[0]), bl = bits_of(mx[1]);
    if (bh + bl <= 8) width = 1;
    else if (bh + bl <= 16) width = 2;
    else if (bh + bl <= 32) width = 4;
    else return false;
    shift = bl;
    pairs->ptr.alloc(static_cast<size_t>(total_out) + 1);
    pairs->codes.alloc(std::max<size_t>(static_cast<size_t>(total_pairs) * width, 1));
    pairs->width = width;
    pairs->shift = shift;
    set_last(pairs->ptr.p + total_out, static_cast<int32_t>(total_pairs), s);
  }
  if (nrows > 0 && (total_out > 0 || pairs)) {
    int32_t* pp = pairs ? pairs->ptr.p : nullptr;
    uint8_t* codes = pairs ? pairs->codes.p : nullptr;
#define BLK_FILL(U, W)                                                                                          \
  do {                                                                                                          \
    prod_sort_kernel<U, false, W><<<sgrid, 64, lds, s>>>(nrows, x_rp, x_ci, y_rp, y_ci, p2cap, ncand.p, nullptr, \
                                                           out.rp.p, out.ci.p, coff.p, pp, codes, shift);       \
    if (nlong > 0)                                                                                              \
      long_emit_kernel<false, W><<<lgrid, 64, 0, s>>>(nlong, lrows.p, loff.p, lsorted.p, lpay.p, nullptr,        \
                                                      out.rp.p, out.ci.p, coff.p, pp, codes, shift);            \
  } while (0)
    if (upper) {
      if (width == 1) BLK_FILL(true, 1); else if (width == 2) BLK_FILL(true, 2); else BLK_FILL(true, 4);
    } else {
      if (width == 1) BLK_FILL(false, 1); else if (width == 2) BLK_FILL(false, 2); else BLK_FILL(false, 4);
    }
#undef BLK_FILL
    HIP_CHECK(hipGetLastError());
  }
  HIP_CHECK(hipStreamSynchronize(s));
  return true;
}

// Workgroup tables of one pass: first rows, lane order, LDS capacity (99.5th
// percentile of the X entries a workgroup spans, within kLdsBytes).
void group_tables(const Product& o, const PairList& pl, int nrows, const int32_t* x_rp, int per, bool by_count,
                  size_t per_entry_bytes, DevBuf<int32_t>& row0, DevBuf<uint8_t>& perm, int& cap, hipStream_t s) {
  const int64_t nout = o.nout;
  const int ngroups = static_cast<int>((nout + per - 1) / per);
  row0.alloc(static_cast<size_t>(ngroups) + 1);
  first_rows_kernel<<<(ngroups + 1 + 255) / 256, 256, 0, s>>>(ngroups, nrows, o.rp.p, per, row0.p);
  HIP_CHECK(hipGetLastError());
  perm.alloc(std::max<size_t>(static_cast<size_t>(nout), 1));
  if (ngroups > 0) {
    group_order_kernel<<<ngroups, 256, 0, s>>>(nout, pl.ptr.p, per, by_count ? 1 : 0, perm.p);
    HIP_CHECK(hipGetLastError());
  }
  std::vector<int32_t> nk;
  if (ngroups > 0) {
    DevBuf<int32_t> dnk(static_cast<size_t>(ngroups));
    group_extent_kernel<<<(ngroups + 255) / 256, 256, 0, s>>>(ngroups, nrows, row0.p, x_rp, dnk.p);
    HIP_CHECK(hipGetLastError());
    nk = download(dnk.p, dnk.n, s);
    nk.erase(std::remove(nk.begin(), nk.end(), -1), nk.end());
  }
  cap = 1;
  if (!nk.empty()) {
    const size_t q = std::min(nk.size() - 1, (nk.size() * 995) / 1000);
    std::nth_element(nk.begin(), nk.begin() + q, nk.end());
    cap = nk[q];
  }
  const int lim = static_cast<int>((kLdsBytes - 16) / per_entry_bytes);
  cap = std::max(1, std::min(cap, lim));
}

}  // namespace

bool structural_product_device(int32_t nrows, int32_t ncols, const int32_t* x_rp, const int32_t* x_ci,
                               const int32_t* y_rp, const int32_t* y_ci, DevBuf<int32_t>& out_rp,
                               DevBuf<int32_t>& out_ci, int64_t& nnz, hipStream_t s) {
  Product o;
  if (!product(nrows, ncols, x_rp, x_ci, y_rp, y_ci, false, nullptr, o, s)) return false;
  nnz = o.nout;
  out_rp = std::move(o.rp);
  out_ci = std::move(o.ci);
  return true;
}

bool ptap_symbolic_device(const bsr_s* A, const bsr_s* P, const bsr_s* R, PtapPlan& plan, bool ap_sort,
                          bool c_sort, DevBuf<int32_t>& c_rowptr, DevBuf<int32_t>& c_colidx, int64_t& c_nnzb,
                          hipStream_t s) {
  // A P (every product column an output)
  Product ap;
  PairList ap_pairs;
  if (!product(A->nbr, P->nbc, A->rowptr, A->colidx, P->rowptr, P->colidx, false, &ap_pairs, ap, s)) return false;
  // the coarse pattern R (A P), and the outputs of the R AP pass
  Product cfull, cup;
  PairList c_pairs;
  if (plan.sym) {
    if (!product(R->nbr, P->nbc, R->rowptr, R->colidx, ap.rp.p, ap.ci.p, false, nullptr, cfull, s)) return false;
    if (!product(R->nbr, P->nbc, R->rowptr, R->colidx, ap.rp.p, ap.ci.p, true, &c_pairs, cup, s)) return false;
    DevBuf<int32_t> uidx(static_cast<size_t>(std::max<int64_t>(cup.nout, 1)));
    DevBuf<int32_t> mir(static_cast<size_t>(std::max<int64_t>(cup.nout, 1)));
    DevBuf<int> ok(1);
    const int one = 1;
    HIP_CHECK(hipMemcpyAsync(ok.p, &one, sizeof(int), hipMemcpyHostToDevice, s));
    if (R->nbr > 0) {
      sym_lists_kernel<<<(R->nbr + 255) / 256, 256, 0, s>>>(R->nbr, cfull.rp.p, cfull.ci.p, cup.rp.p, cup.ci.p,
                                                             uidx.p, mir.p, ok.p);
      HIP_CHECK(hipGetLastError());
    }
    int h = 0;
    HIP_CHECK(hipMemcpyAsync(&h, ok.p, sizeof(int), hipMemcpyDeviceToHost, s));
    HIP_CHECK(hipStreamSynchronize(s));
    BLK_REQUIRE(h == 1, BLKAMG_EINVAL, "coarse pattern is not symmetric");
    plan.c_nslots = cup.nout;
    plan.c_up_idx = std::move(uidx);
    plan.c_mirror = std::move(mir);
  } else {
    if (!product(R->nbr, P->nbc, R->rowptr, R->colidx, ap.rp.p, ap.ci.p, false, &c_pairs, cfull, s)) return false;
  }
  const Product& cout_ = plan.sym ? cup : cfull;
  const int ap_spw = kBlock / plan.ap_nl, c_spw = kBlock / plan.c_nl;
  group_tables(ap, ap_pairs, A->nbr, A->rowptr, ap_spw, ap_sort,
               4 + static_cast<size_t>(A->br) * A->br * dtype_size(A->dtype), plan.ap_slot_row0, plan.ap_perm,
               plan.ap_cap, s);
  group_tables(cout_, c_pairs, R->nbr, R->rowptr, c_spw, c_sort, 4, plan.c_slot_row0, plan.c_perm, plan.c_cap, s);
  HIP_CHECK(hipStreamSynchronize(s));
  plan.ap_nslots = ap.nout;
  plan.ap_pairs = std::move(ap_pairs);
  plan.c_pairs = std::move(c_pairs);
  if (plan.sym) plan.c_up_rp = std::move(cup.rp);
  plan.ap_rowptr = std::move(ap.rp);
  plan.ap_colidx = std::move(ap.ci);
  c_nnzb = cfull.nout;
  c_rowptr = std::move(cfull.rp);
  c_colidx = std::move(cfull.ci);
  return true;
}

}  // namespace blk

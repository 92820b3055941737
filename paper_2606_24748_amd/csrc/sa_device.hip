// Tentative prolongator on the device (paper §2.2 near-null space and tentative
// interpolation; §6, the device-resident cold setup): per aggregate g, the rows of
// the near-null space B of its members, stacked in ascending node order, are
// factored B_g = Q_g R_g by a thin Householder QR with diag(R_g) > 0; the members'
// rows of P~ are the rows of Q_g (bs x nc blocks in column g), and R_g is the coarse
// near-null space of aggregate g.
//
// Members are grouped by a stable radix sort of the aggregate ids (equal ids keep
// ascending node order).  One 64-lane workgroup factors one aggregate with its
// column-major m x nc matrix and the Householder vectors in LDS; every reduction is
// a wave shuffle tree, so the results are deterministic.
#include <algorithm>
#include <string>

#include <hipcub/hipcub.hpp>

#include "internal.hpp"

namespace blk {
namespace {

constexpr int kNc = 6;  // six rigid-body modes

__device__ __forceinline__ double wave_sum(double v) { return group_sum<64>(v); }

__global__ void iota_kernel(int n, int32_t* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = i;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
}

// Boundaries of the sorted aggregate ids: start[g] = first position holding g (ids
// are 0..n_agg-1 after the -1 entries; every aggregate is non-empty).  An id at or
// above n_agg ends the last aggregate early: start[n_agg] is then its position, below
// n, which the host rejects.  Writes stay inside start[0..n_agg].
__global__ void agg_starts_kernel(int n, const int32_t* __restrict__ sorted_agg, int32_t n_agg,
                                  int32_t* __restrict__ start) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int32_t g = sorted_agg[i];
  if (g < 0) return;
  const int32_t prev = i > 0 ? sorted_agg[i - 1] : -1;
  const int32_t top = g < n_agg ? g : n_agg;
  for (int32_t h = prev + 1; h <= top; ++h) start[h] = i;  // ids without members would get a start too
  if (i == n - 1 && g < n_agg)
    for (int32_t h = g + 1; h <= n_agg; ++h) start[h] = n;
}

// One aggregate per 64-lane workgroup.  LDS: Mc [m_cap][kNc] and V [m_cap][kNc],
// column-major with leading dimension m.
__global__ __launch_bounds__(64) void tentative_qr_kernel(int bs, const int32_t* __restrict__ start,
                                                          const int32_t* __restrict__ members,
                                                          const double* __restrict__ B, int m_cap, double tol,
                                                          double* __restrict__ Pt, double* __restrict__ Bc,
                                                          int* __restrict__ flag) {
  extern __shared__ double lds[];
  const int g = blockIdx.x;
  const int lane = threadIdx.x;
  const int s0 = start[g];
  const int cnt = start[g + 1] - s0;
  const int m = cnt * bs;
  if (m < kNc || m > m_cap) {  // too small for the near-null space (or beyond the LDS sizing)
    if (lane == 0) atomicMax(flag, 1);
    return;
  }
  double* Mc = lds;
  double* V = lds + static_cast<size_t>(m_cap) * kNc;
  double amax = 0.0;
  for (int idx = lane; idx < m * kNc; idx += 64) {
    const int c = idx / m, r = idx - c * m;
    const int node = members[s0 + r / bs];
    const double v = B[(static_cast<size_t>(node) * bs + r % bs) * kNc + c];
    Mc[c * m + r] = v;
    amax = fmax(amax, fabs(v));
  }
  const double scale = wave_max(amax);
  __syncthreads();
  double beta[kNc];
  for (int k = 0; k < kNc; ++k) {
    double p = 0.0;
    for (int i = k + lane; i < m; i += 64) p += Mc[k * m + i] * Mc[k * m + i];
    const double nrm = sqrt(wave_sum(p));
    const double head = Mc[k * m + k];
    const double alpha = head >= 0 ? -nrm : nrm;
    double q = 0.0;
    for (int i = lane; i < m; i += 64) {
      const double v = i < k ? 0.0 : (i == k ? head - alpha : Mc[k * m + i]);
      V[k * m + i] = v;
      q += v * v;
    }
    const double vv = wave_sum(q);
    beta[k] = vv > 0 ? 2.0 / vv : 0.0;
    __syncthreads();
    for (int j = k; j < kNc; ++j) {
      double d = 0.0;
      for (int i = k + lane; i < m; i += 64) d += V[k * m + i] * Mc[j * m + i];
      d = wave_sum(d) * beta[k];
      for (int i = k + lane; i < m; i += 64) Mc[j * m + i] -= d * V[k * m + i];
      __syncthreads();
    }
  }
  // R (upper triangle of the reduced matrix) and its signs
  double R[kNc * kNc];
  bool ok = true;
#pragma unroll
  for (int r = 0; r < kNc; ++r)
#pragma unroll
    for (int c = 0; c < kNc; ++c) R[r * kNc + c] = c >= r ? Mc[c * m + r] : 0.0;
#pragma unroll
  for (int r = 0; r < kNc; ++r) ok = ok && fabs(R[r * kNc + r]) > tol * fmax(1.0, scale);
  if (!ok) {
    if (lane == 0) atomicMax(flag, 2);
    return;
  }
  __syncthreads();
  // Q = H_0 ... H_(kNc-1) applied to the first kNc columns of the identity (in Mc)
  for (int idx = lane; idx < m * kNc; idx += 64) {
    const int c = idx / m, r = idx - c * m;
    Mc[c * m + r] = r == c ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int k = kNc - 1; k >= 0; --k) {
    for (int c = 0; c < kNc; ++c) {
      double d = 0.0;
      for (int i = k + lane; i < m; i += 64) d += V[k * m + i] * Mc[c * m + i];
      d = wave_sum(d) * beta[k];
      for (int i = k + lane; i < m; i += 64) Mc[c * m + i] -= d * V[k * m + i];
      __syncthreads();
    }
  }
  double sgn[kNc];
#pragma unroll
  for (int r = 0; r < kNc; ++r) sgn[r] = R[r * kNc + r] < 0 ? -1.0 : 1.0;
  for (int idx = lane; idx < m * kNc; idx += 64) {
    const int r = idx / kNc, c = idx - r * kNc;  // row-major walk of the m x kNc block column
    const int node = members[s0 + r / bs];
    Pt[(static_cast<size_t>(node) * bs + r % bs) * kNc + c] = sgn[c] * Mc[c * m + r];
  }
  if (lane < kNc * kNc) {
    const int r = lane / kNc;
    Bc[static_cast<size_t>(g) * kNc * kNc + lane] = sgn[r] * R[lane];
  }
}

__global__ void rigid_body_kernel(int n, const double* __restrict__ coords, double* __restrict__ B) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double x = coords[3 * i], y = coords[3 * i + 1], z = coords[3 * i + 2];
  // rows c = 0..2 of node i, columns t_x, t_y, t_z, r_z = (-y, x, 0), r_x = (0, -z, y), r_y = (z, 0, -x)
  const double v[18] = {1, 0, 0, -y, 0, z,  //
                        0, 1, 0, x, -z, 0,  //
                        0, 0, 1, 0, y, -x};
  double* o = B + static_cast<size_t>(i) * 18;
#pragma unroll
  for (int t = 0; t < 18; ++t) o[t] = v[t];
}

}  // namespace

// The six rigid-body modes of nodes at d_coords ([n][3]) as d_B [n][3][6].
void rigid_body_modes_device(int32_t n, const double* d_coords, double* d_B, hipStream_t s) {
  if (n <= 0) return;
  rigid_body_kernel<<<(n + 255) / 256, 256, 0, s>>>(n, d_coords, d_B);
  HIP_CHECK(hipGetLastError());
}

// P~ and the coarse near-null space on the device.  d_agg: int32[nbr] (-1 =
// unaggregated, rows of P~ left zero); d_B: double [nbr][bs][kNc]; d_Pt: double
// [nbr][bs][kNc] (every row written); d_Bc: double [n_agg][kNc][kNc].  Sync (one
// flag read).  Fails with EINVAL on an aggregate with fewer than kNc rows or a
// rank-deficient near-null space, like the host version.  Returns false, with
// nothing computed, when an aggregate is too large for the kernel's LDS (64 KiB:
// 682 rows of B); the caller then factors on the host.
bool tentative_device(int32_t nbr, int32_t bs, const int32_t* d_agg, int32_t n_agg, const double* d_B, double* d_Pt,
                      double* d_Bc, hipStream_t s) {
  BLK_REQUIRE(bs >= 1 && bs <= 8, BLKAMG_EINVAL, "block size out of range");
  if (nbr == 0 || n_agg == 0) {
    if (nbr > 0) HIP_CHECK(hipMemsetAsync(d_Pt, 0, static_cast<size_t>(nbr) * bs * kNc * sizeof(double), s));
    return true;
  }
  // stable sort of (agg, node): members of each aggregate in ascending node order
  DevBuf<int32_t> idx(static_cast<size_t>(nbr)), sagg(static_cast<size_t>(nbr)), members(static_cast<size_t>(nbr));
  DevBuf<int32_t> start(static_cast<size_t>(n_agg) + 1);
  DevBuf<int> flag(1);
  iota_kernel<<<(nbr + 255) / 256, 256, 0, s>>>(nbr, idx.p);
  HIP_CHECK(hipGetLastError());
  size_t tmp_bytes = 0;
  HIP_CHECK(hipcub::DeviceRadixSort::SortPairs(nullptr, tmp_bytes, d_agg, sagg.p, idx.p, members.p, nbr, 0, 32, s));
  DevBuf<char> tmp(std::max<size_t>(tmp_bytes, 1));
  HIP_CHECK(hipcub::DeviceRadixSort::SortPairs(tmp.p, tmp_bytes, d_agg, sagg.p, idx.p, members.p, nbr, 0, 32, s));
  // signed keys: the -1 entries (unaggregated) come first; starts are found among the ids
  HIP_CHECK(hipMemsetAsync(start.p, 0xFF, start.bytes(), s));
  agg_starts_kernel<<<(nbr + 255) / 256, 256, 0, s>>>(nbr, sagg.p, n_agg, start.p);
  HIP_CHECK(hipGetLastError());
  std::vector<int32_t> st = download(start.p, start.n, s);
  int32_t m_max = 0;
  BLK_REQUIRE(st[n_agg] == nbr, BLKAMG_EINVAL, "aggregate id at or above n_agg");
  for (int32_t g = 0; g < n_agg; ++g) {
    BLK_REQUIRE(st[g] >= 0 && st[g + 1] >= st[g], BLKAMG_EINVAL, "aggregate ids must be 0..n_agg-1, each used");
    m_max = std::max(m_max, (st[g + 1] - st[g]) * bs);
  }
  const size_t lds = 2 * static_cast<size_t>(m_max) * kNc * sizeof(double);
  if (lds > 64 * 1024) return false;
  HIP_CHECK(hipMemsetAsync(d_Pt, 0, static_cast<size_t>(nbr) * bs * kNc * sizeof(double), s));
  HIP_CHECK(hipMemsetAsync(flag.p, 0, sizeof(int), s));
  tentative_qr_kernel<<<n_agg, 64, lds, s>>>(bs, start.p, members.p, d_B, m_max, 1e-10, d_Pt, d_Bc, flag.p);
  HIP_CHECK(hipGetLastError());
  int h = 0;
  HIP_CHECK(hipMemcpyAsync(&h, flag.p, sizeof(int), hipMemcpyDeviceToHost, s));
  HIP_CHECK(hipStreamSynchronize(s));
  BLK_REQUIRE(h != 1, BLKAMG_EINVAL, "an aggregate is too small for the near-null space");
  BLK_REQUIRE(h != 2, BLKAMG_EINVAL, "an aggregate's near-null space is rank deficient");
  return true;
}

}  // namespace blk

using namespace blk;

extern "C" {

int sa_tentative_device(int32_t nbr, int32_t bs, const int32_t* d_agg, int32_t n_agg, const double* d_B,
                        double* d_Pt, double* d_Bc, void* stream) {
  BLK_API_BEGIN
  BLK_REQUIRE(nbr >= 0 && n_agg >= 0, BLKAMG_EINVAL, "negative size");
  BLK_REQUIRE(nbr == 0 || (d_agg && d_B && d_Pt), BLKAMG_EINVAL, "NULL argument");
  BLK_REQUIRE(n_agg == 0 || d_Bc, BLKAMG_EINVAL, "d_Bc is NULL");
  BLK_REQUIRE(tentative_device(nbr, bs, d_agg, n_agg, d_B, d_Pt, d_Bc, as_stream(stream)), BLKAMG_EINVAL,
              "an aggregate is too large for the device QR (more than 682 rows of the near-null space)");
  BLK_API_END
}

}  // extern "C"

// Finite-element assembly of trilinear hexahedral elasticity on the device: the
// element stiffness kernel and two ways to sum its blocks into a block matrix
// (paper §5: finite-element assembly is the blocked COO primitive's immediate use
// beyond the Galerkin product).
//
// One 64-lane wave per element, lane 8a + b computes the 3x3 block K_ab.  Lanes 0..7
// first evaluate the isoparametric Jacobian at Gauss point q = lane (J^-1 and the
// weighted determinant go to LDS, 80 doubles per element).  The block is then
//   * written to the blocked COO value stream (element-major, (a, b) order), which
//     coo_assemble_blocked sums deterministically (fe_stream_kernel), or
//   * added straight into the matrix at a slot precomputed on the host
//     (element-by-element assembly, fe_q1_kernel), with hardware FP64 atomics, or in
//     colour passes whose elements share no node, so that plain read-modify-writes
//     cannot race and the summation order is fixed.
// Both kernels form every physical gradient with the same expression and sum the
// Gauss points in the same order, so the two routes give the same block values.
#include <algorithm>

#include "internal.hpp"

struct fe_plan_s {
  int64_t n_elem = 0;
  int32_t nbr = 0;
  int64_t nnzb = 0;
  blk::DevBuf<int32_t> slot;       // [n_elem * 64] block of A for (e, a, b), -1 if dropped
  blk::DevBuf<int32_t> dir_slot;   // diagonal block of each Dirichlet node
  blk::DevBuf<int32_t> order;      // elements sorted by colour
  std::vector<int64_t> color_off;  // colour c owns order[color_off[c] .. color_off[c+1])
};

namespace blk {
namespace {

constexpr int kFeWaves = 4;  // elements per 256-thread workgroup
constexpr int kFeGeo = 10;   // per Gauss point: J^-1 (row-major) and det(J) / 8
#ifndef BLK_FE_QUNROLL
#define BLK_FE_QUNROLL 2
#endif
// Gauss points per loop trip of the element-by-element kernel.  Two keep it at about 90
// VGPRs (5 waves per SIMD to cover the latency of the dependent node and coordinate
// loads) instead of ~130 (3 waves) fully unrolled.
constexpr int kFeQUnroll = BLK_FE_QUNROLL;

enum FeMode { kStream = 0, kAtomic = 1, kPlain = 2 };

// d N_a / d xi at xi for the trilinear shape function of local node a (bit 0: x, 1: y, 2: z)
__device__ __forceinline__ void ref_grad(int a, double x, double y, double z, double g[3]) {
  const bool ox = a & 1, oy = (a >> 1) & 1, oz = (a >> 2) & 1;
  const double fx = ox ? x : 1.0 - x, fy = oy ? y : 1.0 - y, fz = oz ? z : 1.0 - z;
  g[0] = (ox ? 1.0 : -1.0) * fy * fz;
  g[1] = fx * (oy ? 1.0 : -1.0) * fz;
  g[2] = fx * fy * (oz ? 1.0 : -1.0);
}

__device__ __forceinline__ double gauss_coord(int bit) {
  // two-point Gauss-Legendre on [0, 1]: 1/2 -+ 1/(2 sqrt 3)
  constexpr double h = 0.28867513459481288225;
  return bit ? 0.5 + h : 0.5 - h;
}

// Jacobian of the element at reference point (x, y, z): G[0..8] = J^-1 (row-major) and
// G[9] = det(J) / 8, the Gauss weight of the 2x2x2 rule on [0, 1]^3 times det(J)
__device__ __forceinline__ void jacobian_point(const int32_t* __restrict__ nodes, const double* __restrict__ coords,
                                               double x, double y, double z, double* G) {
  double J[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};  // J[r * 3 + k] = d x_r / d xi_k
  for (int n = 0; n < 8; ++n) {
    const double* X = coords + static_cast<int64_t>(nodes[n]) * 3;
    double g[3];
    ref_grad(n, x, y, z, g);
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int k = 0; k < 3; ++k) J[r * 3 + k] += X[r] * g[k];
  }
  const double c00 = J[4] * J[8] - J[5] * J[7], c01 = J[5] * J[6] - J[3] * J[8], c02 = J[3] * J[7] - J[4] * J[6];
  const double det = J[0] * c00 + J[1] * c01 + J[2] * c02;
  const double r = 1.0 / det;
  // inverse = adjugate / det, adjugate = transposed cofactor matrix
  G[0] = c00 * r;
  G[1] = (J[2] * J[7] - J[1] * J[8]) * r;
  G[2] = (J[1] * J[5] - J[2] * J[4]) * r;
  G[3] = c01 * r;
  G[4] = (J[0] * J[8] - J[2] * J[6]) * r;
  G[5] = (J[2] * J[3] - J[0] * J[5]) * r;
  G[6] = c02 * r;
  G[7] = (J[1] * J[6] - J[0] * J[7]) * r;
  G[8] = (J[0] * J[4] - J[1] * J[3]) * r;
  G[9] = det * 0.125;
}

// physical gradient: g_c = sum_k (dN/dxi_k) (J^-1)[k][c]
__device__ __forceinline__ void phys_grad(const double rg[3], const double* G, double* g) {
#pragma unroll
  for (int c = 0; c < 3; ++c) g[c] = rg[0] * G[c] + rg[1] * G[3 + c] + rg[2] * G[6 + c];
}

// S += w det(J) g_a g_b^T at one point
__device__ __forceinline__ void add_point(double wd, const double* ga, const double* gb, double S[9]) {
  const double b0 = gb[0], b1 = gb[1], b2 = gb[2];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const double wa = wd * ga[c];
    S[c * 3 + 0] += wa * b0;
    S[c * 3 + 1] += wa * b1;
    S[c * 3 + 2] += wa * b2;
  }
}

// lambda and mu are constant on the element, so with S = sum_q w det(J) g_a g_b^T the
// block is  lambda S + mu (S^T + tr(S) I): one outer product per point
__device__ __forceinline__ void element_block(double l, double m, const double S[9], double K[9]) {
  const double mt = m * (S[0] + S[4] + S[8]);
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int d = 0; d < 3; ++d) K[c * 3 + d] = l * S[c * 3 + d] + m * S[d * 3 + c] + (c == d ? mt : 0.0);
}

// Each wave owns its element and its part of LDS, so a wave barrier orders the LDS
// phases; no workgroup barrier couples the four waves.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Stream mode.  After the Jacobians, lane 8n + q forms the physical gradient of shape
// function n at Gauss point q once, so the per-block loop over the points only forms
// outer products (about a third of the FP64 work of forming both gradients in every
// lane).  One LDS buffer per wave holds the geometry and the gradients, then the 64
// output blocks, which leave as one contiguous 4.6 KB run of 16-byte non-temporal
// stores: the stream is read back only by the assembly, long after.
// 128^3 distorted elements: 2.2 ms against 3.4 ms for the block-per-lane gradients
// with workgroup barriers and plain stores.
__global__ __launch_bounds__(256) void fe_stream_kernel(int64_t count, const int32_t* __restrict__ elem_nodes,
                                                        const double* __restrict__ coords,
                                                        const double* __restrict__ lam,
                                                        const double* __restrict__ mu, double* __restrict__ out) {
  constexpr int kGradOff = 8 * kFeGeo;  // geometry [8][kFeGeo], then gradients [q][n][3]
  static_assert(kGradOff + 8 * 8 * 3 <= 64 * 9, "geometry and gradients fit in the block buffer");
  __shared__ __align__(16) double buf[kFeWaves][64 * 9];
  const int w = static_cast<int>(threadIdx.x) / 64, lane = static_cast<int>(threadIdx.x) % 64;
  const int64_t e = static_cast<int64_t>(blockIdx.x) * kFeWaves + w;
  if (e >= count) return;
  double* geo = buf[w];
  double* grad = buf[w] + kGradOff;
  if (lane < 8) {
    const double x = gauss_coord(lane & 1), y = gauss_coord((lane >> 1) & 1), z = gauss_coord((lane >> 2) & 1);
    jacobian_point(elem_nodes + e * 8, coords, x, y, z, geo + lane * kFeGeo);
  }
  wave_sync();
  {
    const int n = lane >> 3, q = lane & 7;
    double rg[3];
    ref_grad(n, gauss_coord(q & 1), gauss_coord((q >> 1) & 1), gauss_coord((q >> 2) & 1), rg);
    phys_grad(rg, geo + q * kFeGeo, grad + (q * 8 + n) * 3);
  }
  wave_sync();
  const int a = lane >> 3, b = lane & 7;
  double S[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
  for (int q = 0; q < 8; ++q)
    add_point(geo[q * kFeGeo + 9], grad + (q * 8 + a) * 3, grad + (q * 8 + b) * 3, S);
  double K[9];
  element_block(lam[e], mu[e], S, K);
  wave_sync();  // every lane has read the gradients before the blocks overwrite them
#pragma unroll
  for (int t = 0; t < 9; ++t) buf[w][lane * 9 + t] = K[t];
  wave_sync();
  using v2 = double __attribute__((ext_vector_type(2)));
  const v2* src = reinterpret_cast<const v2*>(buf[w]);
  v2* dst = reinterpret_cast<v2*>(out + e * 64 * 9);
  for (int k = lane; k < 64 * 9 / 2; k += 64) __builtin_nontemporal_store(src[k], dst + k);
}

// Element-by-element modes: the same arithmetic, with each lane forming the gradients
// of its own two shape functions at every point and adding its block at its slot.
template <int kMode>
__global__ __launch_bounds__(256) void fe_q1_kernel(int64_t count, const int32_t* __restrict__ order,
                                                    const int32_t* __restrict__ elem_nodes,
                                                    const double* __restrict__ coords, const double* __restrict__ lam,
                                                    const double* __restrict__ mu, const int32_t* __restrict__ slot,
                                                    double* __restrict__ out) {
  static_assert(kMode == kAtomic || kMode == kPlain, "element-by-element modes only");
  __shared__ double geo[kFeWaves][8][kFeGeo];
  const int w = static_cast<int>(threadIdx.x) / 64, lane = static_cast<int>(threadIdx.x) % 64;
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * kFeWaves + w;
  const bool live = idx < count;
  const int64_t e = live ? (order ? order[idx] : idx) : 0;
  if (live && lane < 8) {
    const double x = gauss_coord(lane & 1), y = gauss_coord((lane >> 1) & 1), z = gauss_coord((lane >> 2) & 1);
    jacobian_point(elem_nodes + e * 8, coords, x, y, z, geo[w][lane]);
  }
  __syncthreads();
  if (!live) return;
  const int a = lane >> 3, b = lane & 7;
  double S[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll kFeQUnroll
  for (int q = 0; q < 8; ++q) {
    const double* G = geo[w][q];
    const double x = gauss_coord(q & 1), y = gauss_coord((q >> 1) & 1), z = gauss_coord((q >> 2) & 1);
    double ra[3], rb[3], ga[3], gb[3];
    ref_grad(a, x, y, z, ra);
    ref_grad(b, x, y, z, rb);
    phys_grad(ra, G, ga);
    phys_grad(rb, G, gb);
    add_point(G[9], ga, gb, S);
  }
  double K[9];
  element_block(lam[e], mu[e], S, K);
  const int s = slot[e * 64 + lane];
  if (s >= 0) {
    double* o = out + static_cast<int64_t>(s) * 9;
#pragma unroll
    for (int t = 0; t < 9; ++t) {
      if constexpr (kMode == kAtomic) unsafeAtomicAdd(o + t, K[t]);
      else o[t] += K[t];
    }
  }
}

__global__ void fe_identity_kernel(int64_t n, double* __restrict__ out) {
  const int64_t g = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (g < n * 9) {
    const int t = static_cast<int>(g % 9);
    out[g] = (t == 0 || t == 4 || t == 8) ? 1.0 : 0.0;
  }
}

// zero the values of A, then identity on the Dirichlet diagonal blocks
__global__ void fe_zero_kernel(int64_t n, double* __restrict__ v) {
  const int64_t g = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (g < n) v[g] = 0.0;
}

__global__ void fe_dirichlet_kernel(int32_t n, const int32_t* __restrict__ dslot, double* __restrict__ v) {
  const int64_t g = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (g < static_cast<int64_t>(n) * 9) {
    const int t = static_cast<int>(g % 9);
    v[static_cast<int64_t>(dslot[g / 9]) * 9 + t] = (t == 0 || t == 4 || t == 8) ? 1.0 : 0.0;
  }
}

int64_t grid_of(int64_t count) { return (count + kFeWaves - 1) / kFeWaves; }

template <int kMode>
void launch_fe(int64_t count, const int32_t* order, const int32_t* elem_nodes, const double* coords,
               const double* lam, const double* mu, const int32_t* slot, double* out, hipStream_t s) {
  if (count <= 0) return;
  const int64_t grid = grid_of(count);
  BLK_REQUIRE(grid <= INT32_MAX, BLKAMG_EINVAL, "too many elements for one launch");
  if constexpr (kMode == kStream)
    fe_stream_kernel<<<static_cast<int>(grid), 256, 0, s>>>(count, elem_nodes, coords, lam, mu, out);
  else
    fe_q1_kernel<kMode><<<static_cast<int>(grid), 256, 0, s>>>(count, order, elem_nodes, coords, lam, mu, slot, out);
  HIP_CHECK(hipGetLastError());
}

int32_t find_block(const bsr_s* A, int32_t row, int32_t col) {
  const int32_t* b = A->h_colidx.data() + A->h_rowptr[row];
  const int32_t* end = A->h_colidx.data() + A->h_rowptr[row + 1];
  const int32_t* it = std::lower_bound(b, end, col);
  return (it != end && *it == col) ? static_cast<int32_t>(it - A->h_colidx.data()) : -1;
}

}  // namespace
}  // namespace blk

using namespace blk;

extern "C" {

int fe_q1_stream(int64_t n_elem, const int32_t* d_elem_nodes, const double* d_coords, const double* d_lam,
                 const double* d_mu, int64_t n_identity, double* d_out, void* stream) {
  BLK_API_BEGIN
  BLK_REQUIRE(n_elem >= 0 && n_identity >= 0, BLKAMG_EINVAL, "negative size");
  BLK_REQUIRE(d_out != nullptr || n_elem + n_identity == 0, BLKAMG_EINVAL, "d_out is NULL");
  BLK_REQUIRE(n_elem == 0 || (d_elem_nodes && d_coords && d_lam && d_mu), BLKAMG_EINVAL, "NULL element input");
  BLK_REQUIRE(n_elem == 0 || reinterpret_cast<uintptr_t>(d_out) % 16 == 0, BLKAMG_EINVAL,
              "d_out must be 16-byte aligned (the element blocks leave in 16-byte stores)");
  hipStream_t s = as_stream(stream);
  launch_fe<kStream>(n_elem, nullptr, d_elem_nodes, d_coords, d_lam, d_mu, nullptr, d_out, s);
  if (n_identity > 0) {
    const int64_t tot = n_identity * 9;
    fe_identity_kernel<<<static_cast<int>((tot + 255) / 256), 256, 0, s>>>(n_identity, d_out + n_elem * 64 * 9);
    HIP_CHECK(hipGetLastError());
  }
  BLK_API_END
}

int fe_ebe_plan_create(bsr_t A, int64_t n_elem, const int32_t* h_elem_nodes, const uint8_t* h_dirichlet,
                       fe_plan_t* out) {
  BLK_API_BEGIN
  BLK_REQUIRE(out != nullptr && A != nullptr, BLKAMG_EINVAL, "NULL argument");
  *out = nullptr;
  BLK_REQUIRE(A->dtype == BLKAMG_F64 && A->br == 3 && A->bc == 3 && A->nbr == A->nbc, BLKAMG_EINVAL,
              "A must be square with 3x3 F64 blocks");
  BLK_REQUIRE(n_elem >= 0 && (n_elem == 0 || h_elem_nodes != nullptr), BLKAMG_EINVAL, "bad element list");
  BLK_REQUIRE(n_elem <= INT32_MAX, BLKAMG_EINVAL, "too many elements");
  ensure_host_pattern(A);
  auto P = std::make_unique<fe_plan_s>();
  P->n_elem = n_elem;
  P->nbr = A->nbr;
  P->nnzb = A->nnzb;
  const int32_t nn = A->nbr;
  auto dir = [&](int32_t v) { return h_dirichlet != nullptr && h_dirichlet[v] != 0; };
  std::vector<int32_t> slot(static_cast<size_t>(n_elem) * 64);
  for (int64_t e = 0; e < n_elem; ++e) {
    const int32_t* en = h_elem_nodes + e * 8;
    for (int a = 0; a < 8; ++a) {
      BLK_REQUIRE(en[a] >= 0 && en[a] < nn, BLKAMG_EINVAL, "element node out of range");
      for (int b = 0; b < 8; ++b) {
        int32_t k = -1;
        if (!dir(en[a]) && !dir(en[b])) {
          k = find_block(A, en[a], en[b]);
          BLK_REQUIRE(k >= 0, BLKAMG_EINVAL, "the pattern of A lacks an element coupling");
        }
        slot[e * 64 + a * 8 + b] = k;
      }
    }
  }
  std::vector<int32_t> dslot;
  if (h_dirichlet)
    for (int32_t v = 0; v < nn; ++v)
      if (h_dirichlet[v]) {
        const int32_t k = find_block(A, v, v);
        BLK_REQUIRE(k >= 0, BLKAMG_EINVAL, "the pattern of A lacks a Dirichlet diagonal block");
        dslot.push_back(k);
      }
  // greedy colouring: each element takes the lowest colour none of its nodes has seen
  std::vector<uint64_t> seen(static_cast<size_t>(nn), 0);
  std::vector<uint8_t> color(static_cast<size_t>(n_elem));
  int n_colors = 0;
  for (int64_t e = 0; e < n_elem; ++e) {
    const int32_t* en = h_elem_nodes + e * 8;
    uint64_t used = 0;
    for (int a = 0; a < 8; ++a) used |= seen[en[a]];
    BLK_REQUIRE(~used != 0, BLKAMG_EINVAL, "more than 64 element colours");
    const int c = __builtin_ctzll(~used);
    color[e] = static_cast<uint8_t>(c);
    n_colors = std::max(n_colors, c + 1);
    for (int a = 0; a < 8; ++a) seen[en[a]] |= uint64_t{1} << c;
  }
  P->color_off.assign(static_cast<size_t>(n_colors) + 1, 0);
  for (int64_t e = 0; e < n_elem; ++e) P->color_off[color[e] + 1]++;
  for (int c = 0; c < n_colors; ++c) P->color_off[c + 1] += P->color_off[c];
  std::vector<int32_t> order(static_cast<size_t>(n_elem));
  {
    std::vector<int64_t> next(P->color_off.begin(), P->color_off.end() - 1);
    for (int64_t e = 0; e < n_elem; ++e) order[next[color[e]]++] = static_cast<int32_t>(e);
  }
  upload(P->slot, slot);
  upload(P->dir_slot, dslot);
  upload(P->order, order);
  *out = P.release();
  BLK_API_END
}

int fe_ebe_plan_info(fe_plan_t P, int32_t* n_colors, int64_t* slot_bytes) {
  BLK_API_BEGIN
  BLK_REQUIRE(P != nullptr, BLKAMG_EINVAL, "P is NULL");
  if (n_colors) *n_colors = static_cast<int32_t>(P->color_off.size()) - 1;
  if (slot_bytes) *slot_bytes = static_cast<int64_t>(P->slot.bytes() + P->dir_slot.bytes() + P->order.bytes());
  BLK_API_END
}

int fe_ebe_plan_destroy(fe_plan_t P) {
  BLK_API_BEGIN
  delete P;
  BLK_API_END
}

int fe_q1_assemble_ebe(fe_plan_t P, bsr_t A, const int32_t* d_elem_nodes, const double* d_coords,
                       const double* d_lam, const double* d_mu, int mode, void* stream) {
  BLK_API_BEGIN
  BLK_REQUIRE(P != nullptr && A != nullptr, BLKAMG_EINVAL, "NULL argument");
  BLK_REQUIRE(A->nbr == P->nbr && A->nnzb == P->nnzb && A->dtype == BLKAMG_F64 && A->br == 3 && A->bc == 3,
              BLKAMG_EINVAL, "A does not match the plan");
  BLK_REQUIRE(mode == BLKAMG_FE_ATOMIC || mode == BLKAMG_FE_COLORED, BLKAMG_EINVAL, "bad mode");
  BLK_REQUIRE(P->n_elem == 0 || (d_elem_nodes && d_coords && d_lam && d_mu), BLKAMG_EINVAL, "NULL element input");
  hipStream_t s = as_stream(stream);
  auto* v = static_cast<double*>(A->val);
  const int64_t nv = A->nnzb * 9;
  if (nv > 0) {
    fe_zero_kernel<<<static_cast<int>((nv + 255) / 256), 256, 0, s>>>(nv, v);
    HIP_CHECK(hipGetLastError());
  }
  const int32_t nd = static_cast<int32_t>(P->dir_slot.n);
  if (nd > 0) {
    fe_dirichlet_kernel<<<static_cast<int>((static_cast<int64_t>(nd) * 9 + 255) / 256), 256, 0, s>>>(
        nd, P->dir_slot.p, v);
    HIP_CHECK(hipGetLastError());
  }
  if (mode == BLKAMG_FE_ATOMIC) {
    launch_fe<kAtomic>(P->n_elem, nullptr, d_elem_nodes, d_coords, d_lam, d_mu, P->slot.p, v, s);
  } else {
    for (size_t c = 0; c + 1 < P->color_off.size(); ++c) {
      const int64_t b = P->color_off[c], n = P->color_off[c + 1] - b;
      launch_fe<kPlain>(n, P->order.p + b, d_elem_nodes, d_coords, d_lam, d_mu, P->slot.p, v, s);
    }
  }
  A->stamp++;
  BLK_API_END
}

}  // extern "C"

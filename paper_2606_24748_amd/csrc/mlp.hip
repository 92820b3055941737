// Eigenbound network 12 -> 64 -> 64 -> 2 (ReLU, FP32): forward, loss gradient and
// Adam step.  Every product runs on the matrix cores: one wave computes a 16 x 16
// tile of C with v_mfma_f32_16x16x4_f32, K advancing by 4 per instruction; the
// operands are read straight from global memory (the matrices are at most
// 2000 x 64), and transposed operands are addressed through strides, so the
// backward products need no transposition pass.  Reductions are fixed-order.
#include "mlp.hpp"

namespace blk {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));

// C(i, j) = [C(i, j) +] sum_k A(i, k) B(k, j) [+ bias(j)], then [relu], then
// [0 where mask(i, j) <= 0], with A(i, k) = A[i * a_rs + k * a_cs] and
// B(k, j) = B[k * b_rs + j * b_cs].
struct GemmArgs {
  int M, N, K;
  const float* A;
  int a_rs, a_cs;
  const float* B;
  int b_rs, b_cs;
  float* C;
  int ldc;
  const float* bias;
  const float* mask;
  int m_ld;
  int relu;
  int accumulate;
};

// Lane l of the wave supplies A(i0 + l % 16, k0 + l / 16) and B(k0 + l / 16, j0 + l % 16)
// and receives C(i0 + 4 (l / 16) + r, j0 + l % 16) in accumulator r = 0..3.
__global__ __launch_bounds__(256) void gemm_mfma_kernel(GemmArgs g) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int tiles_n = (g.N + 15) / 16;
  const int tile = blockIdx.x * 4 + wave;
  if (tile >= ((g.M + 15) / 16) * tiles_n) return;  // whole wave
  const int i0 = (tile / tiles_n) * 16, j0 = (tile % tiles_n) * 16;
  const int li = lane & 15, lk = lane >> 4;
  const int ia = i0 + li, jb = j0 + li;
  f4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll 4
  for (int k0 = 0; k0 < g.K; k0 += 4) {
    const int k = k0 + lk;
    const float a = (ia < g.M && k < g.K) ? g.A[static_cast<size_t>(ia) * g.a_rs + static_cast<size_t>(k) * g.a_cs] : 0.f;
    const float b = (k < g.K && jb < g.N) ? g.B[static_cast<size_t>(k) * g.b_rs + static_cast<size_t>(jb) * g.b_cs] : 0.f;
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc, 0, 0, 0);
  }
  const int j = j0 + li;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int i = i0 + 4 * lk + r;
    if (i >= g.M || j >= g.N) continue;
    const size_t o = static_cast<size_t>(i) * g.ldc + j;
    float v = acc[r];
    if (g.accumulate) v += g.C[o];
    if (g.bias) v += g.bias[j];
    if (g.relu) v = fmaxf(v, 0.f);
    if (g.mask && !(g.mask[static_cast<size_t>(i) * g.m_ld + j] > 0.f)) v = 0.f;
    g.C[o] = v;
  }
}

void gemm(const GemmArgs& g, hipStream_t s) {
  if (g.M <= 0 || g.N <= 0) return;
  const int tiles = ((g.M + 15) / 16) * ((g.N + 15) / 16);
  gemm_mfma_kernel<<<(tiles + 3) / 4, 256, 0, s>>>(g);
  HIP_CHECK(hipGetLastError());
}

GemmArgs plain(int M, int N, int K, const float* A, int a_rs, int a_cs, const float* B, int b_rs, int b_cs, float* C,
               int ldc) {
  GemmArgs g{};
  g.M = M;
  g.N = N;
  g.K = K;
  g.A = A;
  g.a_rs = a_rs;
  g.a_cs = a_cs;
  g.B = B;
  g.b_rs = b_rs;
  g.b_cs = b_cs;
  g.C = C;
  g.ldc = ldc;
  return g;
}

// dY = (Y - T) / n ; loss partial per block
__global__ __launch_bounds__(256) void loss_grad_kernel(int n, const float* __restrict__ y, const float* __restrict__ t,
                                                        float* __restrict__ dy, double* __restrict__ loss) {
  __shared__ double lds[4];
  double acc = 0.0;
  for (int e = threadIdx.x; e < n * kMlpOut; e += 256) {
    const double d = static_cast<double>(y[e]) - static_cast<double>(t[e]);
    dy[e] = static_cast<float>(d / n);
    acc += d * d;
  }
  const double s = block_sum_256(acc, lds);
  if (threadIdx.x == 0 && loss) *loss = 0.5 * s / n;
}

// out[j] = sum_i X[i][j] over n rows (one block per column, fixed tree)
__global__ __launch_bounds__(256) void colsum_kernel(int n, int cols, const float* __restrict__ x,
                                                     float* __restrict__ out) {
  __shared__ double lds[4];
  const int j = blockIdx.x;
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) acc += x[static_cast<size_t>(i) * cols + j];
  const double s = block_sum_256(acc, lds);
  if (threadIdx.x == 0) out[j] = static_cast<float>(s);
}

__global__ void adam_kernel(int np, float* __restrict__ th, const float* __restrict__ g, float* __restrict__ m,
                            float* __restrict__ v, float lr, float b1, float b2, float eps, float c1, float c2) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= np) return;
  const float gk = g[k];
  const float mk = b1 * m[k] + (1.f - b1) * gk;
  const float vk = b2 * v[k] + (1.f - b2) * gk * gk;
  m[k] = mk;
  v[k] = vk;
  th[k] -= lr * (mk / c1) / (sqrtf(vk / c2) + eps);
}

}  // namespace

void mlp_forward_dev(const float* th, const float* x, int n, float* h1, float* h2, float* y, hipStream_t s) {
  GemmArgs g = plain(n, kMlpHid, kMlpIn, x, kMlpIn, 1, th + kOffW1, kMlpHid, 1, h1, kMlpHid);
  g.bias = th + kOffB1;
  g.relu = 1;
  gemm(g, s);
  g = plain(n, kMlpHid, kMlpHid, h1, kMlpHid, 1, th + kOffW2, kMlpHid, 1, h2, kMlpHid);
  g.bias = th + kOffB2;
  g.relu = 1;
  gemm(g, s);
  g = plain(n, kMlpOut, kMlpHid, h2, kMlpHid, 1, th + kOffW3, kMlpOut, 1, y, kMlpOut);
  g.bias = th + kOffB3;
  gemm(g, s);
}

}  // namespace blk

using namespace blk;

extern "C" {

int mlp_gemm_f32(int32_t trans_a, int32_t trans_b, int32_t m, int32_t n, int32_t k, const float* d_a, int32_t lda,
                 const float* d_b, int32_t ldb, float* d_c, int32_t ldc, void* stream) {
  BLK_API_BEGIN
  BLK_REQUIRE(m >= 0 && n >= 0 && k >= 0, BLKAMG_EINVAL, "negative size");
  if (m == 0 || n == 0) return BLKAMG_OK;
  BLK_REQUIRE(d_c != nullptr && (k == 0 || (d_a != nullptr && d_b != nullptr)), BLKAMG_EINVAL, "NULL argument");
  BLK_REQUIRE(ldc >= n && lda >= (trans_a ? m : k) && ldb >= (trans_b ? k : n), BLKAMG_EINVAL, "bad leading dimension");
  GemmArgs g = plain(m, n, k, d_a, trans_a ? 1 : lda, trans_a ? lda : 1, d_b, trans_b ? 1 : ldb, trans_b ? ldb : 1, d_c,
                     ldc);
  gemm(g, as_stream(stream));
  BLK_API_END
}

int mlp_forward(const float* d_theta, const float* d_x, int32_t n, float* d_h1, float* d_h2, float* d_y,
                void* stream) {
  BLK_API_BEGIN
  BLK_REQUIRE(n >= 0, BLKAMG_EINVAL, "negative n");
  if (n == 0) return BLKAMG_OK;
  BLK_REQUIRE(d_theta && d_x && d_h1 && d_h2 && d_y, BLKAMG_EINVAL, "NULL argument");
  mlp_forward_dev(d_theta, d_x, n, d_h1, d_h2, d_y, as_stream(stream));
  BLK_API_END
}

int mlp_loss_grad(const float* d_theta, const float* d_x, const float* d_h1, const float* d_h2, const float* d_y,
                  const float* d_t, int32_t n, float* d_work, float* d_grad, double* d_loss, void* stream) {
  BLK_API_BEGIN
  BLK_REQUIRE(n >= 1, BLKAMG_EINVAL, "n must be >= 1");
  BLK_REQUIRE(d_theta && d_x && d_h1 && d_h2 && d_y && d_t && d_work && d_grad, BLKAMG_EINVAL, "NULL argument");
  hipStream_t s = as_stream(stream);
  float* dy = d_work;
  float* dh2 = dy + static_cast<size_t>(n) * kMlpOut;
  float* dh1 = dh2 + static_cast<size_t>(n) * kMlpHid;
  const float* th = d_theta;
  loss_grad_kernel<<<1, 256, 0, s>>>(n, d_y, d_t, dy, d_loss);
  HIP_CHECK(hipGetLastError());
  // layer 3: gW3 = H2^T dY, gb3 = colsum dY, dH2 = (dY W3^T) * [H2 > 0]
  gemm(plain(kMlpHid, kMlpOut, n, d_h2, 1, kMlpHid, dy, kMlpOut, 1, d_grad + kOffW3, kMlpOut), s);
  colsum_kernel<<<kMlpOut, 256, 0, s>>>(n, kMlpOut, dy, d_grad + kOffB3);
  GemmArgs g = plain(n, kMlpHid, kMlpOut, dy, kMlpOut, 1, th + kOffW3, 1, kMlpOut, dh2, kMlpHid);
  g.mask = d_h2;
  g.m_ld = kMlpHid;
  gemm(g, s);
  // layer 2
  gemm(plain(kMlpHid, kMlpHid, n, d_h1, 1, kMlpHid, dh2, kMlpHid, 1, d_grad + kOffW2, kMlpHid), s);
  colsum_kernel<<<kMlpHid, 256, 0, s>>>(n, kMlpHid, dh2, d_grad + kOffB2);
  g = plain(n, kMlpHid, kMlpHid, dh2, kMlpHid, 1, th + kOffW2, 1, kMlpHid, dh1, kMlpHid);
  g.mask = d_h1;
  g.m_ld = kMlpHid;
  gemm(g, s);
  // layer 1
  gemm(plain(kMlpIn, kMlpHid, n, d_x, 1, kMlpIn, dh1, kMlpHid, 1, d_grad + kOffW1, kMlpHid), s);
  colsum_kernel<<<kMlpHid, 256, 0, s>>>(n, kMlpHid, dh1, d_grad + kOffB1);
  HIP_CHECK(hipGetLastError());
  BLK_API_END
}

int mlp_adam(float* d_theta, const float* d_grad, float* d_m, float* d_v, int32_t n_params, int32_t step, float lr,
             float beta1, float beta2, float eps, void* stream) {
  BLK_API_BEGIN
  BLK_REQUIRE(d_theta && d_grad && d_m && d_v, BLKAMG_EINVAL, "NULL argument");
  BLK_REQUIRE(n_params >= 0 && step >= 1, BLKAMG_EINVAL, "bad n_params or step");
  if (n_params == 0) return BLKAMG_OK;
  const float c1 = 1.f - std::pow(beta1, static_cast<float>(step));
  const float c2 = 1.f - std::pow(beta2, static_cast<float>(step));
  adam_kernel<<<(n_params + 255) / 256, 256, 0, as_stream(stream)>>>(n_params, d_theta, d_grad, d_m, d_v, lr, beta1,
                                                                     beta2, eps, c1, c2);
  HIP_CHECK(hipGetLastError());
  BLK_API_END
}

}  // extern "C"

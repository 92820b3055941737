// Smoothed-aggregation hierarchy, smoother, V-cycle and preconditioned CG
// (paper §2.1, §2.2, §3.1, §4.1).  Everything in the solve phase runs on the
// device: the Chebyshev / point-block-Jacobi smoother is fused into the SpMV
// kernels, dot products are reduced deterministically in two stages, the
// Lanczos eigen-estimate and its tridiagonal eigenvalue stay on the device, and
// the coarsest level is applied through the inverse of its Cholesky factor.
#include <algorithm>
#include <cmath>

#include "sa_host.hpp"
#include "spmv_core.hpp"

namespace blk {

constexpr int kMaxCheb = 16;
constexpr int kMaxLanczos = 64;

// Per-level device scalars
struct LevelScalars {
  double alpha[kMaxLanczos];
  double beta[kMaxLanczos];
  double lam;                  // lambda_hat
  double coef[1 + 2 * kMaxCheb];  // 1/theta, then (c1, c2) per Chebyshev step
  double tmp[4];
};

// PCG scalars
enum { S_RZ = 0, S_PW, S_ALPHA, S_RR, S_BETA, S_BB, S_FLAG, S_COUNT };

struct Level {
  bsr_s* A = nullptr;                  // level operator (hierarchy dtype)
  std::unique_ptr<bsr_s> A_own;        // owned operator (levels >= 1, or F32 copy of A0)
  std::unique_ptr<bsr_s> P;            // prolongator (p dtype)
  std::vector<int32_t> agg;
  int32_t n_agg = 0;
  DevBuf<char> dinv;                   // [nbr][bs][bs] hierarchy dtype
  DevBuf<int32_t> diag_idx;            // index of the diagonal block of each row
  DevBuf<char> f, x, r, d, d2, out;    // work vectors (hierarchy dtype)
  DevBuf<double> lz[6];                // Lanczos vectors (F64 hierarchies) ...
  DevBuf<float> lzf[6];                // ... or F32
  int n = 0;                           // scalar dofs
};

}  // namespace blk

struct amg_s {
  blkamg_opts o{};
  int T = BLKAMG_F64;                  // hierarchy dtype
  bsr_s* A0 = nullptr;                 // fine operator (F64, borrowed)
  std::vector<std::unique_ptr<blk::Level>> lv;
  blk::DevBuf<blk::LevelScalars> sc;   // one per level
  blk::DevBuf<double> partial;         // block partial sums
  blk::DevBuf<double> partial2;        // first-level chunk sums
  blk::DevBuf<double> pcg_s;           // PCG scalars
  blk::DevBuf<int> flags;              // [0] non-SPD pivot, [1] singular diagonal block
  // coarsest level dense data (F64)
  int nc = 0;
  blk::DevBuf<double> cmat, cY, cYt, cf, ct, cout;
  // PCG work vectors (F64)
  blk::DevBuf<double> pr, pz, pp, pw;
  double* host_s = nullptr;            // pinned mirror of pcg scalars
  ~amg_s() {
    if (host_s) (void)hipHostFree(host_s);
  }
};

namespace blk {
namespace {

// ---------------------------------------------------------------------------
// Deterministic reductions
// ---------------------------------------------------------------------------
enum RedOp { R_STORE = 0, R_SQRT, R_ALPHA, R_BETA };

// first level: workgroup g sums the fixed chunk [g*chunk, (g+1)*chunk) of partials
__global__ __launch_bounds__(256) void reduce_chunks_kernel(const double* __restrict__ partial, int n, int chunk,
                                                            double* __restrict__ out) {
  __shared__ double lds[4];
  const int lo = blockIdx.x * chunk, hi = min(n, lo + chunk);
  double v = 0.0;
  for (int i = lo + threadIdx.x; i < hi; i += 256) v += partial[i];
  const double s = block_sum_256(v, lds);
  if (threadIdx.x == 0) out[blockIdx.x] = s;
}

__global__ __launch_bounds__(256) void reduce_kernel(const double* __restrict__ partial, int n, double* dst, int op,
                                                     double* pcg) {
  __shared__ double lds[4];
  double v = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) v += partial[i];
  const double s = block_sum_256(v, lds);
  if (threadIdx.x == 0) {
    switch (op) {
      case R_STORE: *dst = s; break;
      case R_SQRT: *dst = sqrt(s > 0.0 ? s : 0.0); break;
      case R_ALPHA:  // s = p.w
        pcg[S_PW] = s;
        if (!(s > 0.0)) { pcg[S_FLAG] = 1.0; pcg[S_ALPHA] = 0.0; }
        else pcg[S_ALPHA] = pcg[S_RZ] / s;
        break;
      case R_BETA:  // s = r.z (new)
        pcg[S_BETA] = s / pcg[S_RZ];
        pcg[S_RZ] = s;
        break;
    }
  }
}

// Deterministic sum of n partials (fixed chunking, fixed order), then `op`.
void reduce(amg_s* M, int n, double* dst, int op, hipStream_t s) {
  const double* src = M->partial.p;
  if (n > 4096) {
    const int chunks = 256;
    const int chunk = (n + chunks - 1) / chunks;
    reduce_chunks_kernel<<<chunks, 256, 0, s>>>(M->partial.p, n, chunk, M->partial2.p);
    HIP_CHECK(hipGetLastError());
    src = M->partial2.p;
    n = chunks;
  }
  reduce_kernel<<<1, 256, 0, s>>>(src, n, dst, op, M->pcg_s.p);
  HIP_CHECK(hipGetLastError());
}

// ---------------------------------------------------------------------------
// Block-diagonal inverse (point-block Jacobi, paper §4.1)
// ---------------------------------------------------------------------------
template <int BS, class TM, class TD>
__global__ void dinv_kernel(int nbr, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                            const TM* __restrict__ val, TD* __restrict__ dinv, int32_t* __restrict__ diag_idx,
                            int* flag) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nbr) return;
  int kd = -1;
  for (int k = rp[r]; k < rp[r + 1]; ++k)
    if (ci[k] == r) { kd = k; break; }
  diag_idx[r] = kd;
  double a[BS][2 * BS];
  for (int i = 0; i < BS; ++i)
    for (int j = 0; j < BS; ++j) {
      a[i][j] = kd >= 0 ? static_cast<double>(ld<double>(val + static_cast<size_t>(kd) * BS * BS + i * BS + j)) : 0.0;
      a[i][BS + j] = (i == j) ? 1.0 : 0.0;
    }
  // Gauss-Jordan with partial pivoting
  bool ok = kd >= 0;
  for (int c = 0; c < BS && ok; ++c) {
    int p = c;
    double best = fabs(a[c][c]);
    for (int i = c + 1; i < BS; ++i)
      if (fabs(a[i][c]) > best) { best = fabs(a[i][c]); p = i; }
    if (!(best > 0.0)) { ok = false; break; }
    if (p != c)
      for (int j = 0; j < 2 * BS; ++j) { const double t = a[c][j]; a[c][j] = a[p][j]; a[p][j] = t; }
    const double inv = 1.0 / a[c][c];
    for (int j = 0; j < 2 * BS; ++j) a[c][j] *= inv;
    for (int i = 0; i < BS; ++i) {
      if (i == c) continue;
      const double f = a[i][c];
      if (f != 0.0)
        for (int j = 0; j < 2 * BS; ++j) a[i][j] -= f * a[c][j];
    }
  }
  if (!ok) atomicExch(flag, 1);
  TD* o = dinv + static_cast<size_t>(r) * BS * BS;
  for (int i = 0; i < BS; ++i)
    for (int j = 0; j < BS; ++j) o[i * BS + j] = static_cast<TD>(ok ? a[i][BS + j] : (i == j ? 1.0 : 0.0));
}

// ---------------------------------------------------------------------------
// Row kernels (one thread per block row, NR = 1)
// ---------------------------------------------------------------------------

// u = Dinv f * coef0 (zero-guess start of the Chebyshev smoother)
template <int BS, class TV>
__global__ void cheb0_kernel(int nbr, const TV* __restrict__ f, const TV* __restrict__ dinv,
                             const double* __restrict__ coef, TV* __restrict__ out) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nbr) return;
  using TA = TV;
  const TA it = static_cast<TA>(coef[0]);
  TA fv[BS];
  for (int j = 0; j < BS; ++j) fv[j] = f[static_cast<size_t>(r) * BS + j];
  const TV* D = dinv + static_cast<size_t>(r) * BS * BS;
  for (int i = 0; i < BS; ++i) {
    TA z = 0;
    for (int j = 0; j < BS; ++j) z = fmadd(static_cast<TA>(D[i * BS + j]), fv[j], z);
    out[static_cast<size_t>(r) * BS + i] = z * it;
  }
}

// Lanczos start: v (splitmix64), Dv = diag-block(A) v, partial v.Dv
__device__ __forceinline__ uint64_t splitmix64(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

template <int BS, class TM, class TV>
__global__ __launch_bounds__(256) void lanczos_start_kernel(int nbr, uint64_t seed, const TM* __restrict__ val,
                                                            const int32_t* __restrict__ diag_idx, TV* __restrict__ v,
                                                            TV* __restrict__ Dv, double* __restrict__ partial) {
  __shared__ double lds[4];
  double acc = 0.0;
  for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < nbr; r += gridDim.x * blockDim.x) {
    double vv[BS];
    for (int j = 0; j < BS; ++j) {
      const uint64_t z = splitmix64(seed ^ static_cast<uint64_t>(static_cast<int64_t>(r) * BS + j));
      vv[j] = static_cast<double>(static_cast<TV>(2.0 * (static_cast<double>(z >> 11) * 0x1.0p-53) - 1.0));
      v[static_cast<size_t>(r) * BS + j] = static_cast<TV>(vv[j]);
    }
    const int kd = diag_idx[r];
    for (int i = 0; i < BS; ++i) {
      double sv = 0.0;
      if (kd >= 0)
        for (int j = 0; j < BS; ++j) sv += ld<double>(val + static_cast<size_t>(kd) * BS * BS + i * BS + j) * vv[j];
      const TV st_ = static_cast<TV>(sv);
      Dv[static_cast<size_t>(r) * BS + i] = st_;
      acc += vv[i] * static_cast<double>(st_);
    }
  }
  const double t = block_sum_256(acc, lds);
  if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

// a = a / s, b = b / s  with s = *scal (elementwise, in place into out arrays)
template <class TV>
__global__ void scale2_kernel(size_t n, const TV* __restrict__ a, const TV* __restrict__ b, const double* scal,
                              TV* __restrict__ ao, TV* __restrict__ bo) {
  const size_t g = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x;
  if (g >= n) return;
  double s = *scal;
  if (!(s > 0.0)) s = 1.0;
  const double inv = 1.0 / s;
  ao[g] = static_cast<TV>(static_cast<double>(a[g]) * inv);
  bo[g] = static_cast<TV>(static_cast<double>(b[g]) * inv);
}

// wy -= alpha*y ; wu = Dinv wy ; partial wu.wy
template <int BS, class TV>
__global__ __launch_bounds__(256) void lanczos_orth_kernel(int nbr, const double* alpha_p, const TV* __restrict__ y,
                                                           TV* __restrict__ wy, const TV* __restrict__ dinv,
                                                           TV* __restrict__ wu, double* __restrict__ partial) {
  __shared__ double lds[4];
  double acc = 0.0;
  const double al = *alpha_p;
  for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < nbr; r += gridDim.x * blockDim.x) {
    double w[BS];
    for (int j = 0; j < BS; ++j) {
      const size_t o = static_cast<size_t>(r) * BS + j;
      const TV wt = static_cast<TV>(static_cast<double>(wy[o]) - al * static_cast<double>(y[o]));
      wy[o] = wt;
      w[j] = static_cast<double>(wt);
    }
    const TV* D = dinv + static_cast<size_t>(r) * BS * BS;
    for (int i = 0; i < BS; ++i) {
      double z = 0.0;
      for (int j = 0; j < BS; ++j) z += static_cast<double>(D[i * BS + j]) * w[j];
      const TV zt = static_cast<TV>(z);
      wu[static_cast<size_t>(r) * BS + i] = zt;
      acc += static_cast<double>(zt) * w[i];
    }
  }
  const double t = block_sum_256(acc, lds);
  if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

// SpMV epilogue for Lanczos: wy = A u - beta_prev * y_prev ; partial u.wy
template <class TV, class TA>
struct EpiLanczos {
  static constexpr bool kReduce = true;
  const TV* u;
  const TV* y_prev;
  const double* beta_prev;  // NULL on the first step
  TV* wy;
  double* partial;
  template <int BR, int NR, int G>
  __device__ __forceinline__ RowVals<double, 2 * BR * NR> prefetch(bool active, int row) const {
    RowVals<double, 2 * BR * NR> p;
#pragma unroll
    for (int t = 0; t < 2 * BR * NR; ++t) p.v[t] = 0.0;
    if (active) {
      const size_t b = static_cast<size_t>(row) * (BR * NR);
#pragma unroll
      for (int t = 0; t < BR * NR; ++t) {
        p.v[t] = static_cast<double>(u[b + t]);
        // y_prev is not read on the first step (its buffer holds no data yet)
        if (beta_prev) p.v[BR * NR + t] = static_cast<double>(y_prev[b + t]);
      }
    }
    return p;
  }
  template <int BR, int NR, int G>
  __device__ __forceinline__ double apply(bool active, int row, int lane, const TA (&s)[BR * NR],
                                          const RowVals<double, 2 * BR * NR>& pre) const {
    double acc = 0.0;
    if (active) {
      const double bp = beta_prev ? *beta_prev : 0.0;
#pragma unroll
      for (int l = 0; l < BR * NR; ++l) {
        if ((l % G) != lane) continue;
        const size_t o = static_cast<size_t>(row) * (BR * NR) + l;
        const double w = static_cast<double>(s[l]) - bp * pre.v[BR * NR + l];
        const TV wt = static_cast<TV>(w);
        wy[o] = wt;
        acc += pre.v[l] * static_cast<double>(wt);
      }
    }
    return acc;
  }
};

// Symmetric tridiagonal largest eigenvalue by Sturm-sequence bisection, then the
// Chebyshev coefficients of Saad Alg. 12.1 for [lo*lam, hi*lam].
__global__ void lanczos_finish_kernel(LevelScalars* sc, int k, double user_lam, double lo, double hi, int degree) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double lam;
  if (user_lam > 0.0) {
    lam = user_lam;
  } else {
    int m = k;
    for (int j = 0; j < k - 1; ++j)
      if (!(sc->beta[j] > 0.0)) { m = j + 1; break; }
    double gl = 1e300, gh = -1e300;
    for (int i = 0; i < m; ++i) {
      const double off = (i > 0 ? fabs(sc->beta[i - 1]) : 0.0) + (i < m - 1 ? fabs(sc->beta[i]) : 0.0);
      gl = fmin(gl, sc->alpha[i] - off);
      gh = fmax(gh, sc->alpha[i] + off);
    }
    double a = gl, b = gh;
    for (int it = 0; it < 200; ++it) {
      const double x = 0.5 * (a + b);
      if (x <= a || x >= b) break;
      // number of eigenvalues < x
      int cnt = 0;
      double q = sc->alpha[0] - x;
      if (q < 0) cnt++;
      for (int i = 1; i < m; ++i) {
        const double qq = (q != 0.0) ? q : 1e-300;
        q = sc->alpha[i] - x - sc->beta[i - 1] * sc->beta[i - 1] / qq;
        if (q < 0) cnt++;
      }
      if (cnt == m) b = x; else a = x;
    }
    lam = 0.5 * (a + b);
  }
  sc->lam = lam;
  const double ea = lo * lam, eb = hi * lam;
  const double theta = 0.5 * (eb + ea), delta = 0.5 * (eb - ea);
  const double sigma = theta / delta;
  double rho = 1.0 / sigma;
  sc->coef[0] = 1.0 / theta;
  for (int t = 1; t < degree; ++t) {
    const double rho1 = 1.0 / (2.0 * sigma - rho);
    sc->coef[1 + 2 * (t - 1)] = rho1 * rho;
    sc->coef[2 + 2 * (t - 1)] = 2.0 * rho1 / delta;
    rho = rho1;
  }
}

// ---------------------------------------------------------------------------
// Fused Chebyshev / residual epilogues.  s = A * (gathered vector).
//   RESID : r_out = f - s
//   INITX : r = f - s ; d = Dinv r / theta ; x_out = x_in + d   (writes r, d, x_out)
//   STEP  : r = f - s (f = current r) ; d' = c1 d_in + c2 Dinv r ; x_out = x_in + d'
//           (r_out, d_out optional)
// ---------------------------------------------------------------------------
enum SmoothMode { M_RESID = 0, M_INITX = 1, M_STEP = 2 };

template <int MODE, class TV, class TA>
struct EpiSmooth {
  static constexpr bool kReduce = false;
  const TV* f;
  TV* r_out;
  const TV* d_in;
  TV* d_out;
  const TV* x_in;
  TV* x_out;
  const TV* dinv;
  const double* coef;
  int step;
  double* partial = nullptr;
  // own-row operands: f (BR*NR), d_in (BR*NR), x_in (BR*NR), Dinv (BR*BR)
  template <int BR, int NR, int G>
  __device__ __forceinline__ RowVals<TA, 3 * BR * NR + BR * BR> prefetch(bool active, int row) const {
    constexpr int N = BR * NR;
    RowVals<TA, 3 * N + BR * BR> p;
#pragma unroll
    for (int t = 0; t < 3 * N + BR * BR; ++t) p.v[t] = TA(0);
    if (!active) return p;
    const size_t b = static_cast<size_t>(row) * N;
#pragma unroll
    for (int t = 0; t < N; ++t) p.v[t] = ld<TA>(f + b + t);
    if (MODE == M_STEP) {
#pragma unroll
      for (int t = 0; t < N; ++t) p.v[N + t] = ld<TA>(d_in + b + t);
    }
    if (MODE != M_RESID) {
#pragma unroll
      for (int t = 0; t < N; ++t) p.v[2 * N + t] = ld<TA>(x_in + b + t);
      const TV* D = dinv + static_cast<size_t>(row) * (BR * BR);
#pragma unroll
      for (int t = 0; t < BR * BR; ++t) p.v[3 * N + t] = ld<TA>(D + t);
    }
    return p;
  }
  template <int BR, int NR, int G>
  __device__ __forceinline__ double apply(bool active, int row, int lane, const TA (&s)[BR * NR],
                                          const RowVals<TA, 3 * BR * NR + BR * BR>& pre) const {
    constexpr int N = BR * NR;
    if (!active) return 0.0;
    const size_t base = static_cast<size_t>(row) * N;
    TA r[N];
#pragma unroll
    for (int t = 0; t < N; ++t) r[t] = pre.v[t] - s[t];
    if (MODE == M_RESID) {
#pragma unroll
      for (int l = 0; l < N; ++l)
        if ((l % G) == lane) r_out[base + l] = static_cast<TV>(r[l]);
      return 0.0;
    }
    TA z[N];
#pragma unroll
    for (int i = 0; i < BR; ++i) {
#pragma unroll
      for (int q = 0; q < NR; ++q) z[i * NR + q] = TA(0);
#pragma unroll
      for (int j = 0; j < BR; ++j) {
        const TA dij = pre.v[3 * N + i * BR + j];
#pragma unroll
        for (int q = 0; q < NR; ++q) z[i * NR + q] = fmadd(dij, r[j * NR + q], z[i * NR + q]);
      }
    }
    TA c1 = TA(0), c2;
    if (MODE == M_INITX) {
      c2 = static_cast<TA>(coef[0]);
    } else {
      c1 = static_cast<TA>(coef[1 + 2 * step]);
      c2 = static_cast<TA>(coef[2 + 2 * step]);
    }
#pragma unroll
    for (int l = 0; l < N; ++l) {
      if ((l % G) != lane) continue;
      const size_t o = base + l;
      TA dn = c2 * z[l];
      if (MODE == M_STEP) dn = fmadd(c1, pre.v[N + l], dn);
      x_out[o] = static_cast<TV>(pre.v[2 * N + l] + dn);
      if (r_out) r_out[o] = static_cast<TV>(r[l]);
      if (d_out) d_out[o] = static_cast<TV>(dn);
    }
    return 0.0;
  }
};

// PCG: w = A p, partial p.w
struct EpiPcgW {
  static constexpr bool kReduce = true;
  const double* p;
  double* w;
  double* partial;
  template <int BR, int NR, int G>
  __device__ __forceinline__ RowVals<double, BR * NR> prefetch(bool active, int row) const {
    RowVals<double, BR * NR> pv;
#pragma unroll
    for (int t = 0; t < BR * NR; ++t) pv.v[t] = active ? p[static_cast<size_t>(row) * (BR * NR) + t] : 0.0;
    return pv;
  }
  template <int BR, int NR, int G>
  __device__ __forceinline__ double apply(bool active, int row, int lane, const double (&s)[BR * NR],
                                          const RowVals<double, BR * NR>& pre) const {
    double acc = 0.0;
    if (active) {
#pragma unroll
      for (int l = 0; l < BR * NR; ++l) {
        if ((l % G) != lane) continue;
        const size_t o = static_cast<size_t>(row) * (BR * NR) + l;
        w[o] = s[l];
        acc += pre.v[l] * s[l];
      }
    }
    return acc;
  }
};

// x += alpha p ; r -= alpha w ; partial r.r
__global__ __launch_bounds__(256) void pcg_update_kernel(size_t n, const double* __restrict__ sc,
                                                         const double* __restrict__ p, const double* __restrict__ w,
                                                         double* __restrict__ x, double* __restrict__ r,
                                                         double* __restrict__ partial) {
  __shared__ double lds[4];
  double acc = 0.0;
  const double a = sc[S_ALPHA];
  for (size_t g = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x; g < n;
       g += static_cast<size_t>(gridDim.x) * blockDim.x) {
    x[g] = fmadd(a, p[g], x[g]);
    const double rv = fmadd(-a, w[g], r[g]);
    r[g] = rv;
    acc = fmadd(rv, rv, acc);
  }
  const double t = block_sum_256(acc, lds);
  if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

// partial a.b (and optional copy b -> c)
__global__ __launch_bounds__(256) void dot_kernel(size_t n, const double* __restrict__ a, const double* __restrict__ b,
                                                  double* __restrict__ partial) {
  __shared__ double lds[4];
  double acc = 0.0;
  for (size_t g = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x; g < n;
       g += static_cast<size_t>(gridDim.x) * blockDim.x)
    acc = fmadd(a[g], b[g], acc);
  const double t = block_sum_256(acc, lds);
  if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

// p = z + beta p   (beta_index < 0: p = z)
__global__ void pcg_p_kernel(size_t n, const double* __restrict__ sc, int use_beta, const double* __restrict__ z,
                             double* __restrict__ p) {
  const size_t g = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x;
  if (g >= n) return;
  p[g] = use_beta ? fmadd(sc[S_BETA], p[g], z[g]) : z[g];
}

// r = b, x = 0, partial b.b
__global__ __launch_bounds__(256) void pcg_init_kernel(size_t n, const double* __restrict__ b, double* __restrict__ x,
                                                       double* __restrict__ r, double* __restrict__ partial) {
  __shared__ double lds[4];
  double acc = 0.0;
  for (size_t g = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x; g < n;
       g += static_cast<size_t>(gridDim.x) * blockDim.x) {
    const double v = b[g];
    r[g] = v;
    x[g] = 0.0;
    acc = fmadd(v, v, acc);
  }
  const double t = block_sum_256(acc, lds);
  if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

// ---------------------------------------------------------------------------
// Prolongator smoothing (cold setup, paper §2.2): for row i and column b of P,
//   P_ib = [agg(i) == b] P~_i - omega Dinv_i sum_{j in A_i, agg(j) == b} A_ij P~_j
// ---------------------------------------------------------------------------
template <int BS, int NC>
__global__ void smooth_p_kernel(int nbr, const int32_t* __restrict__ a_rp, const int32_t* __restrict__ a_ci,
                                const double* __restrict__ a_v, const int32_t* __restrict__ agg,
                                const double* __restrict__ pt, const double* __restrict__ dinv,
                                const double* __restrict__ lam, double omega_scale, const int32_t* __restrict__ p_rp,
                                const int32_t* __restrict__ p_ci, double* __restrict__ p_v) {
  const int64_t gidx = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  // one thread per stored block of P: find its row by binary search on p_rp
  const int64_t nnz = p_rp[nbr];
  if (gidx >= nnz) return;
  int lo = 0, hi = nbr;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (p_rp[mid] <= gidx) lo = mid; else hi = mid;
  }
  const int i = lo;
  const int b = p_ci[gidx];
  double acc[BS * NC];
  for (int t = 0; t < BS * NC; ++t) acc[t] = 0.0;
  for (int k = a_rp[i]; k < a_rp[i + 1]; ++k) {
    const int j = a_ci[k];
    if (agg[j] != b) continue;
    const double* ab = a_v + static_cast<size_t>(k) * BS * BS;
    const double* pb = pt + static_cast<size_t>(j) * BS * NC;
    for (int r = 0; r < BS; ++r)
      for (int m = 0; m < BS; ++m) {
        const double a = ab[r * BS + m];
        for (int c = 0; c < NC; ++c) acc[r * NC + c] += a * pb[m * NC + c];
      }
  }
  const double omega = omega_scale / *lam;
  const double* D = dinv + static_cast<size_t>(i) * BS * BS;
  double* o = p_v + static_cast<size_t>(gidx) * BS * NC;
  for (int r = 0; r < BS; ++r)
    for (int c = 0; c < NC; ++c) {
      double z = 0.0;
      for (int m = 0; m < BS; ++m) z += D[r * BS + m] * acc[m * NC + c];
      const double base = (agg[i] == b) ? pt[static_cast<size_t>(i) * BS * NC + r * NC + c] : 0.0;
      o[r * NC + c] = base - omega * z;
    }
}

// ---------------------------------------------------------------------------
// Coarsest level: dense expansion, Cholesky, inverse of the factor
// ---------------------------------------------------------------------------
template <class TM>
__global__ void expand_dense_kernel(int nbr, int bs, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                    const TM* __restrict__ val, double* __restrict__ M, int n) {
  const int r = blockIdx.x;
  if (r >= nbr) return;
  for (int k = rp[r]; k < rp[r + 1]; ++k) {
    const int c = ci[k];
    for (int e = threadIdx.x; e < bs * bs; e += blockDim.x) {
      const int i = e / bs, j = e % bs;
      M[static_cast<size_t>(r * bs + i) * n + c * bs + j] = ld<double>(val + static_cast<size_t>(k) * bs * bs + e);
    }
  }
}

// Blocked dense Cholesky and inverse of the factor (coarsest level, FP64).
// Tiles of kT x kT; the matrix is n x n row-major; tiles that stick out of the
// matrix are padded with the identity on the diagonal and zeros elsewhere.
constexpr int kT = 32;

__device__ __forceinline__ double mat_at(const double* M, int n, int i, int j) {
  if (i < n && j < n) return M[static_cast<size_t>(i) * n + j];
  return (i == j) ? 1.0 : 0.0;
}

// Factor the diagonal tile of panel k in LDS (all threads of the block take part).
__device__ void factor_diag_tile(const double* M, int n, int k, double (*D)[kT + 1], int* flag) {
  const int base = k * kT;
  for (int e = threadIdx.x; e < kT * kT; e += blockDim.x) {
    const int i = e / kT, j = e % kT;
    D[i][j] = mat_at(M, n, base + i, base + j);
  }
  __syncthreads();
  for (int c = 0; c < kT; ++c) {
    if (threadIdx.x == 0) {
      double d = D[c][c];
      if (!(d > 0.0)) { *flag = 1; d = 1.0; }
      D[c][c] = sqrt(d);
    }
    __syncthreads();
    const double piv = D[c][c];
    for (int i = c + 1 + threadIdx.x; i < kT; i += blockDim.x) D[i][c] /= piv;
    __syncthreads();
    for (int e = threadIdx.x; e < kT * kT; e += blockDim.x) {
      const int i = e / kT, j = e % kT;
      if (j > c && i >= j) D[i][j] -= D[i][c] * D[j][c];
    }
    __syncthreads();
  }
}

// Panel k: block 0 writes L_kk; block b > 0 writes L_{k+b,k} = A_{k+b,k} L_kk^-T.
__global__ __launch_bounds__(256) void chol_panel_kernel(double* __restrict__ M, int n, int k, int* flag) {
  __shared__ double D[kT][kT + 1];
  __shared__ double X[kT][kT + 1];
  factor_diag_tile(M, n, k, D, flag);
  const int I = k + static_cast<int>(blockIdx.x);
  const int rb = I * kT, cb = k * kT;
  if (blockIdx.x == 0) {
    for (int e = threadIdx.x; e < kT * kT; e += blockDim.x) {
      const int i = e / kT, j = e % kT;
      if (rb + i < n && cb + j < n) M[static_cast<size_t>(rb + i) * n + cb + j] = (j <= i) ? D[i][j] : 0.0;
    }
    return;
  }
  for (int e = threadIdx.x; e < kT * kT; e += blockDim.x) {
    const int i = e / kT, j = e % kT;
    X[i][j] = mat_at(M, n, rb + i, cb + j);
  }
  __syncthreads();
  // row r of X: x_j = (a_j - sum_{m<j} x_m L_jm) / L_jj
  if (threadIdx.x < kT) {
    const int r = threadIdx.x;
    for (int j = 0; j < kT; ++j) {
      double v = X[r][j];
      for (int m = 0; m < j; ++m) v -= X[r][m] * D[j][m];
      X[r][j] = v / D[j][j];
    }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < kT * kT; e += blockDim.x) {
    const int i = e / kT, j = e % kT;
    if (rb + i < n && cb + j < n) M[static_cast<size_t>(rb + i) * n + cb + j] = X[i][j];
  }
}

// Trailing update after panel k: A_IJ -= L_Ik L_Jk^T for k < J <= I (lower tiles),
// one block per tile; tile index t enumerates the lower triangle of the trailing part.
__global__ __launch_bounds__(256) void chol_update_kernel(double* __restrict__ M, int n, int k, int nt) {
  __shared__ double Li[kT][kT + 1];
  __shared__ double Lj[kT][kT + 1];
  const int m = nt - k - 1;
  int t = blockIdx.x, I = 0;
  while (t >= I + 1) { t -= I + 1; ++I; }  // t-th tile of row I in the lower triangle
  (void)m;
  const int J = t;
  const int ri = (k + 1 + I) * kT, rj = (k + 1 + J) * kT, cb = k * kT;
  for (int e = threadIdx.x; e < kT * kT; e += blockDim.x) {
    const int i = e / kT, j = e % kT;
    Li[i][j] = (ri + i < n && cb + j < n) ? M[static_cast<size_t>(ri + i) * n + cb + j] : 0.0;
    Lj[i][j] = (rj + i < n && cb + j < n) ? M[static_cast<size_t>(rj + i) * n + cb + j] : 0.0;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < kT * kT; e += blockDim.x) {
    const int i = e / kT, j = e % kT;
    if (ri + i >= n || rj + j >= n) continue;
    double sdot = 0.0;
#pragma unroll 8
    for (int q = 0; q < kT; ++q) sdot += Li[i][q] * Lj[j][q];
    M[static_cast<size_t>(ri + i) * n + rj + j] -= sdot;
  }
}

// Inverse of the lower factor, block row I: Y_IJ = L_II^-1 (delta_IJ - sum_{K=J}^{I-1} L_IK Y_KJ),
// one block per J <= I.
__global__ __launch_bounds__(256) void tri_inverse_row_kernel(const double* __restrict__ L, double* __restrict__ Y,
                                                              int n, int I) {
  __shared__ double Dd[kT][kT + 1];
  __shared__ double S[kT][kT + 1];
  __shared__ double A[kT][kT + 1];
  __shared__ double Bt[kT][kT + 1];
  const int J = blockIdx.x;
  const int ri = I * kT, cj = J * kT;
  for (int e = threadIdx.x; e < kT * kT; e += blockDim.x) {
    const int i = e / kT, j = e % kT;
    Dd[i][j] = mat_at(L, n, ri + i, ri + j);
    S[i][j] = (I == J && i == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int K = J; K < I; ++K) {
    const int rk = K * kT;
    for (int e = threadIdx.x; e < kT * kT; e += blockDim.x) {
      const int i = e / kT, j = e % kT;
      A[i][j] = (ri + i < n && rk + j < n) ? L[static_cast<size_t>(ri + i) * n + rk + j] : 0.0;
      Bt[i][j] = (rk + i < n && cj + j < n) ? Y[static_cast<size_t>(rk + i) * n + cj + j] : 0.0;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < kT * kT; e += blockDim.x) {
      const int i = e / kT, j = e % kT;
      double sdot = 0.0;
#pragma unroll 8
      for (int q = 0; q < kT; ++q) sdot += A[i][q] * Bt[q][j];
      S[i][j] -= sdot;
    }
    __syncthreads();
  }
  // forward substitution L_II y = s, column j by thread j
  if (threadIdx.x < kT) {
    const int j = threadIdx.x;
    for (int i = 0; i < kT; ++i) {
      double v = S[i][j];
      for (int q = 0; q < i; ++q) v -= Dd[i][q] * S[q][j];
      S[i][j] = v / Dd[i][i];
    }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < kT * kT; e += blockDim.x) {
    const int i = e / kT, j = e % kT;
    if (ri + i < n && cj + j < n) Y[static_cast<size_t>(ri + i) * n + cj + j] = S[i][j];
  }
}

__global__ void transpose_dense_kernel(const double* __restrict__ A, double* __restrict__ B, int n) {
  const size_t e = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x;
  if (e >= static_cast<size_t>(n) * n) return;
  const int i = static_cast<int>(e / n), j = static_cast<int>(e % n);
  B[static_cast<size_t>(j) * n + i] = A[e];
}

// y = M x for a dense row-major matrix whose row i is nonzero only in [lo_i, hi_i):
// lower (lo=0, hi=i+1) or upper (lo=i, hi=n).  One wave per row.
template <class TI, class TO>
__global__ __launch_bounds__(256) void dense_tri_matvec_kernel(const double* __restrict__ M, int n, int upper,
                                                               const TI* __restrict__ x, TO* __restrict__ y) {
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= n) return;
  const int lo = upper ? row : 0, hi = upper ? n : row + 1;
  double s = 0.0;
  for (int k = lo + lane; k < hi; k += 64) s += M[static_cast<size_t>(row) * n + k] * static_cast<double>(x[k]);
  s = group_sum<64>(s);
  if (lane == 0) y[row] = static_cast<TO>(s);
}

template <class TI, class TO>
__global__ void cast_vec_kernel(size_t n, const TI* __restrict__ a, TO* __restrict__ b) {
  const size_t g = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x;
  if (g < n) b[g] = static_cast<TO>(a[g]);
}

inline int vgrid(size_t n) { return static_cast<int>((n + 255) / 256); }
// grid of a reducing grid-stride kernel: at most 2048 workgroups (= partial sums)
inline int rgrid(size_t n) { return static_cast<int>(std::max<size_t>(1, std::min<size_t>((n + 255) / 256, 2048))); }

// ---------------------------------------------------------------------------
// Host-side drivers
// ---------------------------------------------------------------------------

template <class TV>
TV* buf(DevBuf<char>& b) { return reinterpret_cast<TV*>(b.p); }

template <class TV>
void smooth_launch_resid(const bsr_s* A, const TV* x_gather, const TV* f, TV* r_out, hipStream_t s);

template <int BS, int MODE, class TV>
void launch_smooth(const bsr_s* A, const TV* gather, const EpiSmooth<MODE, TV, TV>& epi, hipStream_t s) {
  launch_rows<BS, BS, 1, TV, TV, TV>(lanes_for(A), A->nbr, A->rowptr, A->colidx, static_cast<const TV*>(A->val),
                                      gather, epi, s);
}

template <int MODE, class TV>
void smooth(const bsr_s* A, const TV* gather, const EpiSmooth<MODE, TV, TV>& epi, hipStream_t s) {
  if (A->br == 3) launch_smooth<3, MODE, TV>(A, gather, epi, s);
  else launch_smooth<6, MODE, TV>(A, gather, epi, s);
}

size_t tsize(int T) { return T == BLKAMG_F64 ? 8 : 4; }

void alloc_level_vectors(amg_s* M, Level& L, bool coarsest) {
  const size_t n = static_cast<size_t>(L.A->nbr) * L.A->br;
  L.n = static_cast<int>(n);
  const size_t b = n * tsize(M->T);
  L.f.alloc(b);
  L.out.alloc(b);
  if (!coarsest) {
    L.x.alloc(b);
    L.r.alloc(b);
    L.d.alloc(b);
    L.d2.alloc(b);
  }
}

// Block-diagonal inverse of level l into L.dinv (hierarchy dtype).
void compute_dinv(amg_s* M, Level& L, hipStream_t s) {
  const bsr_s* A = L.A;
  const int bs = A->br;
  if (!L.dinv.p) {
    L.dinv.alloc(static_cast<size_t>(A->nbr) * bs * bs * tsize(M->T));
    L.diag_idx.alloc(static_cast<size_t>(std::max(A->nbr, 1)));
  }
  const int grid = vgrid(A->nbr);
  if (A->nbr == 0) return;
#define BLK_DINV(BS, TM, TD)                                                                                   \
  dinv_kernel<BS, TM, TD><<<grid, 256, 0, s>>>(A->nbr, A->rowptr, A->colidx, static_cast<const TM*>(A->val),   \
                                                 reinterpret_cast<TD*>(L.dinv.p), L.diag_idx.p, M->flags.p + 1)
  if (M->T == BLKAMG_F64) {
    if (bs == 3) BLK_DINV(3, double, double); else BLK_DINV(6, double, double);
  } else {
    if (bs == 3) BLK_DINV(3, float, float); else BLK_DINV(6, float, float);
  }
#undef BLK_DINV
  HIP_CHECK(hipGetLastError());
}

// k-step Lanczos on D^-1 A in the D inner product; result into sc[l].
template <class TV>
void lanczos_typed(amg_s* M, int l, hipStream_t s) {
  Level& L = *M->lv[l];
  const bsr_s* A = L.A;
  const int bs = A->br;
  const int nbr = A->nbr;
  const size_t n = static_cast<size_t>(nbr) * bs;
  TV* V[6];
  for (int t = 0; t < 6; ++t) {
    if constexpr (sizeof(TV) == 8) {
      if (!L.lz[t].p) L.lz[t].alloc(n);
      V[t] = reinterpret_cast<TV*>(L.lz[t].p);
    } else {
      if (!L.lzf[t].p) L.lzf[t].alloc(n);
      V[t] = reinterpret_cast<TV*>(L.lzf[t].p);
    }
  }
  // roles: u_prev, u, wu, y_prev, y, wy
  int iu_prev = 0, iu = 1, iwu = 2, iy_prev = 3, iy = 4, iwy = 5;
  LevelScalars* sc = M->sc.p + l;
  const int rg = rgrid(nbr);
  // start: v -> (u, y) = (v, Dv) / sqrt(v.Dv)
  if (bs == 3)
    lanczos_start_kernel<3, TV, TV><<<rg, 256, 0, s>>>(nbr, M->o.lanczos_seed + static_cast<uint64_t>(l),
                                                       static_cast<const TV*>(A->val), L.diag_idx.p, V[iwu], V[iwy],
                                                       M->partial.p);
  else
    lanczos_start_kernel<6, TV, TV><<<rg, 256, 0, s>>>(nbr, M->o.lanczos_seed + static_cast<uint64_t>(l),
                                                       static_cast<const TV*>(A->val), L.diag_idx.p, V[iwu], V[iwy],
                                                       M->partial.p);
  HIP_CHECK(hipGetLastError());
  reduce(M, rg, sc->tmp, R_SQRT, s);
  scale2_kernel<TV><<<vgrid(n), 256, 0, s>>>(n, V[iwu], V[iwy], sc->tmp, V[iu], V[iy]);
  HIP_CHECK(hipGetLastError());
  const int k = M->o.lanczos_steps;
  const int G = lanes_for(A);
  const TV* dinv = reinterpret_cast<const TV*>(L.dinv.p);
  for (int step = 0; step < k; ++step) {
    EpiLanczos<TV, TV> epi{V[iu], V[iy_prev], step > 0 ? sc->beta + (step - 1) : nullptr, V[iwy], M->partial.p};
    const int sg =
        bs == 3
            ? launch_rows<3, 3, 1, TV, TV, TV>(G, nbr, A->rowptr, A->colidx, static_cast<const TV*>(A->val), V[iu], epi, s)
            : launch_rows<6, 6, 1, TV, TV, TV>(G, nbr, A->rowptr, A->colidx, static_cast<const TV*>(A->val), V[iu], epi, s);
    reduce(M, sg, sc->alpha + step, R_STORE, s);
    if (step == k - 1) break;
    if (bs == 3)
      lanczos_orth_kernel<3, TV><<<rg, 256, 0, s>>>(nbr, sc->alpha + step, V[iy], V[iwy], dinv, V[iwu], M->partial.p);
    else
      lanczos_orth_kernel<6, TV><<<rg, 256, 0, s>>>(nbr, sc->alpha + step, V[iy], V[iwy], dinv, V[iwu], M->partial.p);
    HIP_CHECK(hipGetLastError());
    reduce(M, rg, sc->beta + step, R_SQRT, s);
    // (u_prev, u) <- (u, wu/beta) ; (y_prev, y) <- (y, wy/beta)
    scale2_kernel<TV><<<vgrid(n), 256, 0, s>>>(n, V[iwu], V[iwy], sc->beta + step, V[iu_prev], V[iy_prev]);
    HIP_CHECK(hipGetLastError());
    std::swap(iu_prev, iu);    // u_prev slot now holds the new u
    std::swap(iy_prev, iy);
  }
}

void refresh_level_scalars(amg_s* M, int l, const double* h_lambda, hipStream_t s) {
  const double user = h_lambda ? h_lambda[l] : 0.0;
  if (!h_lambda) {
    if (M->T == BLKAMG_F64) lanczos_typed<double>(M, l, s);
    else lanczos_typed<float>(M, l, s);
  }
  lanczos_finish_kernel<<<1, 1, 0, s>>>(M->sc.p + l, M->o.lanczos_steps, user, M->o.cheb_lo, M->o.cheb_hi,
                                         M->o.cheb_degree);
  HIP_CHECK(hipGetLastError());
}

void coarse_factor(amg_s* M, hipStream_t s) {
  Level& L = *M->lv.back();
  const bsr_s* A = L.A;
  const int n = A->nbr * A->br;
  M->nc = n;
  if (!M->cmat.p) {
    const size_t nn = static_cast<size_t>(std::max(n, 1)) * std::max(n, 1);
    M->cmat.alloc(nn);
    M->cY.alloc(nn);
    M->cYt.alloc(nn);
    M->cf.alloc(std::max(n, 1));
    M->ct.alloc(std::max(n, 1));
    M->cout.alloc(std::max(n, 1));
  }
  if (n == 0) return;
  HIP_CHECK(hipMemsetAsync(M->cmat.p, 0, static_cast<size_t>(n) * n * sizeof(double), s));
  if (A->dtype == BLKAMG_F64)
    expand_dense_kernel<double><<<A->nbr, 64, 0, s>>>(A->nbr, A->br, A->rowptr, A->colidx,
                                                      static_cast<const double*>(A->val), M->cmat.p, n);
  else
    expand_dense_kernel<float><<<A->nbr, 64, 0, s>>>(A->nbr, A->br, A->rowptr, A->colidx,
                                                     static_cast<const float*>(A->val), M->cmat.p, n);
  HIP_CHECK(hipGetLastError());
  const int nt = (n + kT - 1) / kT;
  HIP_CHECK(hipMemsetAsync(M->cY.p, 0, static_cast<size_t>(n) * n * sizeof(double), s));
  for (int k = 0; k < nt; ++k) {
    chol_panel_kernel<<<nt - k, 256, 0, s>>>(M->cmat.p, n, k, M->flags.p);
    const int m = nt - k - 1;
    if (m > 0) chol_update_kernel<<<m * (m + 1) / 2, 256, 0, s>>>(M->cmat.p, n, k, nt);
  }
  HIP_CHECK(hipGetLastError());
  for (int I = 0; I < nt; ++I) tri_inverse_row_kernel<<<I + 1, 256, 0, s>>>(M->cmat.p, M->cY.p, n, I);
  HIP_CHECK(hipGetLastError());
  transpose_dense_kernel<<<vgrid(static_cast<size_t>(n) * n), 256, 0, s>>>(M->cY.p, M->cYt.p, n);
  HIP_CHECK(hipGetLastError());
}

// z = (L L^T)^-1 f = Y^T (Y f)
template <class TV>
void coarse_apply(amg_s* M, const TV* f, TV* z, hipStream_t s) {
  const int n = M->nc;
  if (n == 0) return;
  const int g = (n + 3) / 4;
  dense_tri_matvec_kernel<TV, double><<<g, 256, 0, s>>>(M->cY.p, n, 0, f, M->ct.p);
  dense_tri_matvec_kernel<double, TV><<<g, 256, 0, s>>>(M->cYt.p, n, 1, M->ct.p, z);
  HIP_CHECK(hipGetLastError());
}

// One V-cycle on level l: z = V(f)
template <class TV>
void vcycle_level(amg_s* M, int l, const TV* f, TV* out, hipStream_t s) {
  if (l == static_cast<int>(M->lv.size()) - 1) {
    coarse_apply<TV>(M, f, out, s);
    return;
  }
  Level& L = *M->lv[l];
  const bsr_s* A = L.A;
  const int nbr = A->nbr;
  const int bs = A->br;
  const TV* dinv = buf<TV>(L.dinv);
  const double* coef = M->sc.p[l].coef;  // device pointer arithmetic on the struct array
  TV* x = buf<TV>(L.x);
  TV* r = buf<TV>(L.r);
  TV* d = buf<TV>(L.d);
  TV* d2 = buf<TV>(L.d2);
  const int k = M->o.cheb_degree;
  // pre-smoothing from a zero guess
  TV* first = (k == 1) ? x : d;
  if (nbr > 0) {
    if (bs == 3) cheb0_kernel<3, TV><<<vgrid(nbr), 256, 0, s>>>(nbr, f, dinv, coef, first);
    else cheb0_kernel<6, TV><<<vgrid(nbr), 256, 0, s>>>(nbr, f, dinv, coef, first);
    HIP_CHECK(hipGetLastError());
  }
  for (int t = 1; t < k; ++t) {
    const bool last = (t == k - 1);
    EpiSmooth<M_STEP, TV, TV> e{t == 1 ? f : r, last ? nullptr : r, d, last ? nullptr : d2, t == 1 ? d : x, x,
                                dinv, coef, t - 1};
    smooth<M_STEP, TV>(A, d, e, s);
    std::swap(d, d2);
  }
  // residual and restriction
  {
    EpiSmooth<M_RESID, TV, TV> e{f, r, nullptr, nullptr, nullptr, nullptr, dinv, coef, 0};
    smooth<M_RESID, TV>(A, x, e, s);
  }
  Level& C = *M->lv[l + 1];
  TV* fc = buf<TV>(C.f);
  TV* oc = buf<TV>(C.out);
  bsr_s* R = transpose_of(L.P.get(), s);
  spmv(R, 1.0, r, 0.0, fc, M->T, 1, s);
  vcycle_level<TV>(M, l + 1, fc, oc, s);
  spmv(L.P.get(), 1.0, oc, 1.0, x, M->T, 1, s);
  // post-smoothing from x
  {
    EpiSmooth<M_INITX, TV, TV> e{f, r, nullptr, d, x, out, dinv, coef, 0};
    smooth<M_INITX, TV>(A, x, e, s);
  }
  for (int t = 1; t < k; ++t) {
    const bool last = (t == k - 1);
    EpiSmooth<M_STEP, TV, TV> e{r, last ? nullptr : r, d, last ? nullptr : d2, out, out, dinv, coef, t - 1};
    smooth<M_STEP, TV>(A, d, e, s);
    std::swap(d, d2);
  }
}

void vcycle(amg_s* M, const double* r, double* z, hipStream_t s) {
  Level& L0 = *M->lv[0];
  const size_t n = static_cast<size_t>(L0.n);
  if (M->T == BLKAMG_F64) {
    vcycle_level<double>(M, 0, r, z, s);
  } else {
    float* f = buf<float>(L0.f);
    float* o = buf<float>(L0.out);
    cast_vec_kernel<double, float><<<vgrid(n), 256, 0, s>>>(n, r, f);
    HIP_CHECK(hipGetLastError());
    vcycle_level<float>(M, 0, f, o, s);
    cast_vec_kernel<float, double><<<vgrid(n), 256, 0, s>>>(n, o, z);
    HIP_CHECK(hipGetLastError());
  }
}

// Host strength mask for epsilon > 0 (block Frobenius norms).
std::vector<uint8_t> strength_mask(bsr_s* A, double eps) {
  ensure_host_pattern(A);
  std::vector<double> v = download(static_cast<const double*>(A->val), static_cast<size_t>(A->nnzb) * A->block_elems());
  const size_t be = A->block_elems();
  std::vector<double> nrm(static_cast<size_t>(A->nnzb)), dn(static_cast<size_t>(A->nbr), 0.0);
  for (int64_t k = 0; k < A->nnzb; ++k) {
    double ss = 0.0;
    for (size_t e = 0; e < be; ++e) ss += v[k * be + e] * v[k * be + e];
    nrm[k] = std::sqrt(ss);
  }
  for (int32_t i = 0; i < A->nbr; ++i)
    for (int32_t k = A->h_rowptr[i]; k < A->h_rowptr[i + 1]; ++k)
      if (A->h_colidx[k] == i) dn[i] = nrm[k];
  std::vector<uint8_t> m(static_cast<size_t>(A->nnzb), 1);
  for (int32_t i = 0; i < A->nbr; ++i)
    for (int32_t k = A->h_rowptr[i]; k < A->h_rowptr[i + 1]; ++k)
      m[k] = nrm[k] >= eps * std::sqrt(dn[i] * dn[A->h_colidx[k]]) ? 1 : 0;
  return m;
}

void check_flags(amg_s* M, hipStream_t s) {
  int h[3];
  HIP_CHECK(hipMemcpyAsync(h, M->flags.p, sizeof(h), hipMemcpyDeviceToHost, s));
  HIP_CHECK(hipStreamSynchronize(s));
  if (h[1]) {
    HIP_CHECK(hipMemsetAsync(M->flags.p, 0, 3 * sizeof(int), s));
    fail(BLKAMG_EINVAL, "a diagonal block is missing or singular");
  }
  if (h[0]) {
    HIP_CHECK(hipMemsetAsync(M->flags.p, 0, 3 * sizeof(int), s));
    fail(BLKAMG_ENOTSPD, "coarsest Cholesky met a non-positive pivot");
  }
}

void smoother_refresh(amg_s* M, const double* h_lambda, hipStream_t s) {
  const int nl = static_cast<int>(M->lv.size());
  for (int l = 0; l < nl - 1; ++l) {
    compute_dinv(M, *M->lv[l], s);
    refresh_level_scalars(M, l, h_lambda, s);
  }
  coarse_factor(M, s);
  check_flags(M, s);
}

void galerkin_recompute(amg_s* M, hipStream_t s) {
  if (M->T != BLKAMG_F64) {
    bsr_s* A0f = M->lv[0]->A;
    cast_values(M->A0->val, BLKAMG_F64, A0f->val, BLKAMG_F32, static_cast<size_t>(M->A0->nnzb) * M->A0->block_elems(), s);
    A0f->stamp++;
  }
  for (size_t l = 0; l + 1 < M->lv.size(); ++l) {
    const int rc = ptap_numeric(M->lv[l]->A, M->lv[l]->P.get(), M->lv[l + 1]->A, s);
    if (rc != BLKAMG_OK) fail(rc, std::string("ptap_numeric: ") + blkamg_last_error());
  }
}

}  // namespace
}  // namespace blk

using namespace blk;

extern "C" {

void blkamg_opts_default(blkamg_opts* o) {
  if (!o) return;
  o->max_levels = 10;
  o->coarse_eq_limit = 1000;
  o->strength_eps = 0.0;
  o->cheb_degree = 2;
  o->cheb_lo = 0.1;
  o->cheb_hi = 1.1;
  o->lanczos_steps = 10;
  o->lanczos_seed = 0x5EED;
  o->omega_scale = 4.0 / 3.0;
  o->hier_dtype = BLKAMG_F64;
  o->p_dtype = BLKAMG_F64;
}

}  // extern "C"

namespace blk {
namespace {

// Copy of a matrix pattern with new (zeroed) values of another dtype.
std::unique_ptr<bsr_s> clone_pattern(bsr_s* A, int dtype) {
  ensure_host_pattern(A);
  return make_owned(A->nbr, A->nbc, A->br, A->bc, dtype, A->h_rowptr, A->h_colidx);
}

Level* get_level(amg_s* M, int32_t l) {
  BLK_REQUIRE(M != nullptr, BLKAMG_EINVAL, "M is NULL");
  BLK_REQUIRE(l >= 0 && l < static_cast<int32_t>(M->lv.size()), BLKAMG_EINVAL, "level out of range");
  return M->lv[l].get();
}

}  // namespace
}  // namespace blk

extern "C" {

int amg_setup(bsr_t A0, const double* h_coords, const uint8_t* h_dirichlet, const blkamg_opts* opts, void* stream,
              amg_t* out) {
  BLK_API_BEGIN
  BLK_REQUIRE(A0 != nullptr && out != nullptr && h_coords != nullptr, BLKAMG_EINVAL, "NULL argument");
  *out = nullptr;
  blkamg_opts o;
  if (opts) o = *opts; else blkamg_opts_default(&o);
  BLK_REQUIRE(A0->dtype == BLKAMG_F64, BLKAMG_EINVAL, "A0 must be F64");
  BLK_REQUIRE(A0->br == 3 && A0->bc == 3 && A0->nbr == A0->nbc, BLKAMG_EINVAL, "A0 must be square with 3x3 blocks");
  BLK_REQUIRE(A0->nbr > 0, BLKAMG_EINVAL, "A0 is empty");
  BLK_REQUIRE(o.max_levels >= 1 && o.cheb_degree >= 1 && o.cheb_degree <= kMaxCheb, BLKAMG_EINVAL,
              "bad max_levels or cheb_degree");
  BLK_REQUIRE(o.lanczos_steps >= 2 && o.lanczos_steps <= kMaxLanczos, BLKAMG_EINVAL, "lanczos_steps must be in 2..64");
  BLK_REQUIRE(o.cheb_lo > 0 && o.cheb_hi > o.cheb_lo && o.omega_scale > 0 && o.strength_eps >= 0, BLKAMG_EINVAL,
              "bad smoother parameters");
  BLK_REQUIRE(o.hier_dtype == BLKAMG_F64 || o.hier_dtype == BLKAMG_F32, BLKAMG_EINVAL, "hier_dtype must be F64 or F32");
  BLK_REQUIRE((o.hier_dtype == BLKAMG_F64 && o.p_dtype == BLKAMG_F64) ||
                  (o.hier_dtype == BLKAMG_F32 && (o.p_dtype == BLKAMG_F32 || o.p_dtype == BLKAMG_BF16)),
              BLKAMG_EINVAL, "p_dtype must be F64 for F64 hierarchies and F32/BF16 for F32 hierarchies");
  hipStream_t s = as_stream(stream);
  HIP_CHECK(hipStreamSynchronize(s));
  auto M = std::make_unique<amg_s>();
  M->o = o;
  M->T = BLKAMG_F64;  // the cold setup runs in F64; an F32 hierarchy is derived at the end
  M->A0 = A0;
  M->flags.alloc(4);
  HIP_CHECK(hipMemset(M->flags.p, 0, 4 * sizeof(int)));
  M->sc.alloc(static_cast<size_t>(o.max_levels));
  HIP_CHECK(hipMemset(M->sc.p, 0, static_cast<size_t>(o.max_levels) * sizeof(LevelScalars)));
  // one partial per block of any reduction launch: at most nbr/4 (4 rows per block)
  M->partial.alloc(static_cast<size_t>(A0->nbr) / 4 + 8192);
  M->partial2.alloc(256);
  M->pcg_s.alloc(S_COUNT);
  HIP_CHECK(hipHostMalloc(reinterpret_cast<void**>(&M->host_s), S_COUNT * sizeof(double)));

  // ---- cold setup in F64 ----
  std::vector<double> B = rigid_body_modes(A0->nbr, h_coords);
  std::vector<uint8_t> dir;
  if (h_dirichlet) dir.assign(h_dirichlet, h_dirichlet + A0->nbr);
  bsr_s* A = A0;
  std::unique_ptr<bsr_s> A_owned;  // owns A when it is a coarse operator
  const int nc_bs = 6;
  while (static_cast<int64_t>(A->nbr) * A->br > o.coarse_eq_limit &&
         static_cast<int>(M->lv.size()) < o.max_levels - 1) {
    ensure_host_pattern(A);
    std::vector<uint8_t> strong;
    if (o.strength_eps > 0) strong = strength_mask(A, o.strength_eps);
    std::vector<int32_t> agg;
    const int32_t n_agg = aggregate_host(A->nbr, A->h_rowptr.data(), A->h_colidx.data(),
                                         dir.empty() ? nullptr : dir.data(), strong.empty() ? nullptr : strong.data(), agg);
    if (n_agg == 0) break;
    std::vector<double> Pt, Bc;
    tentative_host(A->nbr, A->br, nc_bs, agg, n_agg, B, Pt, Bc);
    const int l = static_cast<int>(M->lv.size());
    M->lv.push_back(std::make_unique<Level>());
    Level& Lv = *M->lv.back();
    Lv.A = A;
    Lv.A_own = std::move(A_owned);
    Lv.agg = std::move(agg);
    Lv.n_agg = n_agg;
    compute_dinv(M.get(), Lv, s);
    check_flags(M.get(), s);
    refresh_level_scalars(M.get(), l, nullptr, s);
    // smoothed prolongator: pattern of A P~ on the host, values on the device
    std::vector<int32_t> ptrp(static_cast<size_t>(A->nbr) + 1, 0), ptci;
    for (int32_t i = 0; i < A->nbr; ++i) {
      if (Lv.agg[i] >= 0) ptci.push_back(Lv.agg[i]);
      ptrp[i + 1] = static_cast<int32_t>(ptci.size());
    }
    std::vector<int32_t> prp, pci;
    structural_product_host(A->nbr, A->h_rowptr, A->h_colidx, n_agg, ptrp, ptci, prp, pci);
    Lv.P = make_owned(A->nbr, n_agg, A->br, nc_bs, BLKAMG_F64, std::move(prp), std::move(pci));
    {
      DevBuf<int32_t> dagg;
      upload(dagg, Lv.agg);
      DevBuf<double> dpt;
      upload(dpt, Pt);
      const int64_t nnz = Lv.P->nnzb;
      if (nnz > 0) {
        const int grid = static_cast<int>((nnz + 255) / 256);
        if (A->br == 3)
          smooth_p_kernel<3, 6><<<grid, 256, 0, s>>>(A->nbr, A->rowptr, A->colidx, static_cast<const double*>(A->val),
                                                     dagg.p, dpt.p, reinterpret_cast<const double*>(Lv.dinv.p),
                                                     &M->sc.p[l].lam, o.omega_scale, Lv.P->rowptr, Lv.P->colidx,
                                                     static_cast<double*>(Lv.P->val));
        else
          smooth_p_kernel<6, 6><<<grid, 256, 0, s>>>(A->nbr, A->rowptr, A->colidx, static_cast<const double*>(A->val),
                                                     dagg.p, dpt.p, reinterpret_cast<const double*>(Lv.dinv.p),
                                                     &M->sc.p[l].lam, o.omega_scale, Lv.P->rowptr, Lv.P->colidx,
                                                     static_cast<double*>(Lv.P->val));
        HIP_CHECK(hipGetLastError());
      }
      HIP_CHECK(hipStreamSynchronize(s));  // dagg / dpt are freed at scope exit
    }
    bsr_t C = nullptr;
    int rc = ptap_symbolic_ex(A, Lv.P.get(), BLKAMG_PTAP_SYMMETRIC, &C, stream);
    if (rc != BLKAMG_OK) fail(rc, std::string("ptap_symbolic: ") + blkamg_last_error());
    A_owned.reset(C);
    rc = ptap_numeric(A, Lv.P.get(), C, stream);
    if (rc != BLKAMG_OK) fail(rc, std::string("ptap_numeric: ") + blkamg_last_error());
    A = C;
    B = std::move(Bc);
    dir.clear();
  }
  {
    M->lv.push_back(std::make_unique<Level>());
    Level& Lc = *M->lv.back();
    Lc.A = A;
    Lc.A_own = std::move(A_owned);
  }
  const int nl = static_cast<int>(M->lv.size());

  // ---- derive the F32 hierarchy: A_l and P_l stored in F32 (P optionally BF16) ----
  if (o.hier_dtype == BLKAMG_F32) {
    std::vector<std::unique_ptr<bsr_s>> Af(nl), Pf(nl);
    Af[0] = clone_pattern(A0, BLKAMG_F32);
    cast_values(A0->val, BLKAMG_F64, Af[0]->val, BLKAMG_F32, static_cast<size_t>(A0->nnzb) * 9, s);
    for (int l = 0; l + 1 < nl; ++l) {
      bsr_s* P64 = M->lv[l]->P.get();
      Pf[l] = clone_pattern(P64, o.p_dtype);
      cast_values(P64->val, BLKAMG_F64, Pf[l]->val, o.p_dtype, static_cast<size_t>(P64->nnzb) * P64->block_elems(), s);
      bsr_t C = nullptr;
      int rc = ptap_symbolic_ex(Af[l].get(), Pf[l].get(), BLKAMG_PTAP_SYMMETRIC, &C, stream);
      if (rc != BLKAMG_OK) fail(rc, std::string("ptap_symbolic: ") + blkamg_last_error());
      Af[l + 1].reset(C);
      rc = ptap_numeric(Af[l].get(), Pf[l].get(), C, stream);
      if (rc != BLKAMG_OK) fail(rc, std::string("ptap_numeric: ") + blkamg_last_error());
    }
    HIP_CHECK(hipStreamSynchronize(s));
    for (int l = 0; l < nl; ++l) {
      Level& Lv = *M->lv[l];
      Lv.A_own = std::move(Af[l]);  // frees the F64 coarse operator of this level
      Lv.A = Lv.A_own.get();
      if (l + 1 < nl) Lv.P = std::move(Pf[l]);
      Lv.dinv.release();
      Lv.diag_idx.release();
      for (auto& v : Lv.lz) v.release();
    }
    M->T = BLKAMG_F32;
  }
  for (int l = 0; l < nl; ++l) alloc_level_vectors(M.get(), *M->lv[l], l == nl - 1);
  smoother_refresh(M.get(), nullptr, s);
  HIP_CHECK(hipStreamSynchronize(s));
  *out = M.release();
  BLK_API_END
}

int amg_destroy(amg_t M) {
  BLK_API_BEGIN
  if (M) (void)hipDeviceSynchronize();
  delete M;
  BLK_API_END
}

int amg_num_levels(amg_t M, int32_t* n_levels) {
  BLK_API_BEGIN
  BLK_REQUIRE(M != nullptr && n_levels != nullptr, BLKAMG_EINVAL, "NULL argument");
  *n_levels = static_cast<int32_t>(M->lv.size());
  BLK_API_END
}

int amg_level(amg_t M, int32_t level, bsr_t* A, bsr_t* P) {
  BLK_API_BEGIN
  Level* L = get_level(M, level);
  if (A) *A = L->A;
  if (P) *P = L->P.get();
  BLK_API_END
}

int amg_aggregates(amg_t M, int32_t level, int32_t* h_agg) {
  BLK_API_BEGIN
  Level* L = get_level(M, level);
  BLK_REQUIRE(level + 1 < static_cast<int32_t>(M->lv.size()), BLKAMG_EINVAL, "the coarsest level has no aggregates");
  BLK_REQUIRE(h_agg != nullptr, BLKAMG_EINVAL, "h_agg is NULL");
  std::copy(L->agg.begin(), L->agg.end(), h_agg);
  BLK_API_END
}

int amg_lambdas(amg_t M, double* h_lam) {
  BLK_API_BEGIN
  BLK_REQUIRE(M != nullptr && h_lam != nullptr, BLKAMG_EINVAL, "NULL argument");
  const size_t nl = M->lv.size();
  std::vector<LevelScalars> sc = download(M->sc.p, nl);
  for (size_t l = 0; l + 1 < nl; ++l) h_lam[l] = sc[l].lam;
  BLK_API_END
}

int amg_galerkin_recompute(amg_t M, void* stream) {
  BLK_API_BEGIN
  BLK_REQUIRE(M != nullptr, BLKAMG_EINVAL, "M is NULL");
  galerkin_recompute(M, as_stream(stream));
  BLK_API_END
}

int amg_smoother_refresh(amg_t M, const double* h_lambda, void* stream) {
  BLK_API_BEGIN
  BLK_REQUIRE(M != nullptr, BLKAMG_EINVAL, "M is NULL");
  if (h_lambda)
    for (size_t l = 0; l + 1 < M->lv.size(); ++l)
      BLK_REQUIRE(h_lambda[l] > 0.0, BLKAMG_EINVAL, "lambda must be positive");
  smoother_refresh(M, h_lambda, as_stream(stream));
  BLK_API_END
}

int vcycle_apply(amg_t M, const double* d_r, double* d_z, int32_t nrhs, void* stream) {
  BLK_API_BEGIN
  BLK_REQUIRE(M != nullptr && d_r != nullptr && d_z != nullptr, BLKAMG_EINVAL, "NULL argument");
  BLK_REQUIRE(nrhs == 1, BLKAMG_EINVAL, "vcycle_apply supports nrhs == 1");
  BLK_REQUIRE(d_r != d_z, BLKAMG_EINVAL, "r and z must not alias");
  vcycle(M, d_r, d_z, as_stream(stream));
  BLK_API_END
}

int pcg_solve(bsr_t A, amg_t M, const double* d_b, double* d_x, double rtol, int32_t maxit, int32_t nrhs,
              int32_t* iters, double* relres, void* stream) {
  BLK_API_BEGIN
  BLK_REQUIRE(A != nullptr && M != nullptr && d_b != nullptr && d_x != nullptr, BLKAMG_EINVAL, "NULL argument");
  BLK_REQUIRE(nrhs == 1, BLKAMG_EINVAL, "pcg_solve supports nrhs == 1");
  BLK_REQUIRE(A->dtype == BLKAMG_F64 && A->br == A->bc && A->nbr == A->nbc, BLKAMG_EINVAL, "A must be square F64");
  BLK_REQUIRE(static_cast<int64_t>(A->nbr) * A->br == static_cast<int64_t>(M->lv[0]->n), BLKAMG_EINVAL,
              "A and the hierarchy have different sizes");
  BLK_REQUIRE(A->br == 3 || A->br == 6, BLKAMG_EINVAL, "A must have 3x3 or 6x6 blocks");
  BLK_REQUIRE(maxit >= 0 && rtol >= 0.0, BLKAMG_EINVAL, "bad rtol or maxit");
  hipStream_t s = as_stream(stream);
  const size_t n = static_cast<size_t>(M->lv[0]->n);
  if (M->pr.n < n) {
    HIP_CHECK(hipStreamSynchronize(s));
    M->pr.alloc(n);
    M->pz.alloc(n);
    M->pp.alloc(n);
    M->pw.alloc(n);
  }
  double* r = M->pr.p;
  double* z = M->pz.p;
  double* p = M->pp.p;
  double* w = M->pw.p;
  double* sc = M->pcg_s.p;
  const int vg = rgrid(n);
  HIP_CHECK(hipMemsetAsync(sc, 0, S_COUNT * sizeof(double), s));
  pcg_init_kernel<<<vg, 256, 0, s>>>(n, d_b, d_x, r, M->partial.p);
  HIP_CHECK(hipGetLastError());
  reduce(M, vg, sc + S_BB, R_STORE, s);
  HIP_CHECK(hipMemcpyAsync(M->host_s, sc, S_COUNT * sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_CHECK(hipStreamSynchronize(s));
  const double bn = std::sqrt(M->host_s[S_BB]);
  int32_t it = 0;
  double rn = bn;
  if (iters) *iters = 0;
  if (relres) *relres = 0.0;
  if (bn == 0.0) return BLKAMG_OK;
  vcycle(M, r, z, s);
  dot_kernel<<<vg, 256, 0, s>>>(n, r, z, M->partial.p);
  HIP_CHECK(hipGetLastError());
  reduce(M, vg, sc + S_RZ, R_STORE, s);
  pcg_p_kernel<<<vgrid(n), 256, 0, s>>>(n, sc, 0, z, p);
  HIP_CHECK(hipGetLastError());
  const int G = lanes_for(A);
  bool converged = false;
  while (it < maxit) {
    EpiPcgW epi{p, w, M->partial.p};
    const int sg = A->br == 3 ? launch_rows<3, 3, 1, double, double, double>(G, A->nbr, A->rowptr, A->colidx,
                                                                            static_cast<const double*>(A->val), p, epi, s)
                              : launch_rows<6, 6, 1, double, double, double>(G, A->nbr, A->rowptr, A->colidx,
                                                                            static_cast<const double*>(A->val), p, epi, s);
    reduce(M, sg, nullptr, R_ALPHA, s);
    pcg_update_kernel<<<vg, 256, 0, s>>>(n, sc, p, w, d_x, r, M->partial.p);
    HIP_CHECK(hipGetLastError());
    reduce(M, vg, sc + S_RR, R_STORE, s);
    ++it;
    HIP_CHECK(hipMemcpyAsync(M->host_s, sc, S_COUNT * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_CHECK(hipStreamSynchronize(s));
    if (M->host_s[S_FLAG] != 0.0) {
      if (iters) *iters = it;
      fail(BLKAMG_EBREAKDOWN, "CG breakdown: p^T A p <= 0");
    }
    rn = std::sqrt(M->host_s[S_RR]);
    if (rn <= rtol * bn) { converged = true; break; }
    vcycle(M, r, z, s);
    dot_kernel<<<vg, 256, 0, s>>>(n, r, z, M->partial.p);
    HIP_CHECK(hipGetLastError());
    reduce(M, vg, nullptr, R_BETA, s);
    pcg_p_kernel<<<vgrid(n), 256, 0, s>>>(n, sc, 1, z, p);
    HIP_CHECK(hipGetLastError());
  }
  if (iters) *iters = it;
  if (relres) *relres = rn / bn;
  if (!converged) return BLKAMG_ENOCONV;
  BLK_API_END
}

}  // extern "C"

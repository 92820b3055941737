// Device kernels of the hierarchy, smoother, V-cycle and CG (paper §2.1, §2.2, §3.1,
// §4.1), shared by single-instance and batched solves.
//
// A level of a batch holds several independent instances.  Their block rows are
// contiguous "segments"; the segments that are smoothed (active) come first, the
// ones whose coarsest level this is (terminal) last.  Per-instance quantities
// (Lanczos coefficients, lambda_hat, Chebyshev coefficients, CG scalars) are looked
// up from the row by a binary search of the segment offsets.  All reductions are
// deterministic: fixed chunks summed in a fixed order.
#pragma once

#include <cmath>

#include "spmv_core.hpp"

namespace blk {

constexpr int kMaxCheb = 16;
constexpr int kMaxLanczos = 64;

struct LevelScalars {
  double alpha[kMaxLanczos];
  double beta[kMaxLanczos];
  double lam;                     // lambda_hat
  double coef[1 + 2 * kMaxCheb];  // 1/theta, then (c1, c2) per Chebyshev step
  double tmp[4];
  float coef_f[1 + 2 * kMaxCheb];  // the same coefficients rounded to FP32
};

// Chebyshev coefficient t in the arithmetic type of the smoother
template <class TA>
__device__ __forceinline__ TA cheb_coef(const LevelScalars& S, int t) {
  if constexpr (sizeof(TA) == 4) return S.coef_f[t];
  else return static_cast<TA>(S.coef[t]);
}

// segment of row `row` among off[0..n] (off[0] = 0 <= row < off[n])
__device__ __forceinline__ int seg_of(const int32_t* __restrict__ off, int n, int row) {
  int lo = 0, hi = n;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (off[mid] <= row) lo = mid; else hi = mid;
  }
  return lo;
}

__device__ __forceinline__ uint64_t splitmix64(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// ---------------------------------------------------------------------------
// Segmented dot products.  A chunk is a row range inside one segment; workgroup c
// sums chunk c for every right-hand side q into partial[c * NR + q].
// ---------------------------------------------------------------------------
template <int NR, class T, class TB = T>
__global__ __launch_bounds__(256) void seg_dot_kernel(const T* __restrict__ a, const TB* __restrict__ b,
                                                      const int32_t* __restrict__ lo, const int32_t* __restrict__ hi,
                                                      double* __restrict__ partial) {
  __shared__ double lds[4 * NR];
  const int c = blockIdx.x;
  double acc[NR];
#pragma unroll
  for (int q = 0; q < NR; ++q) acc[q] = 0.0;
  for (int i = lo[c] + threadIdx.x; i < hi[c]; i += 256) {
#pragma unroll
    for (int q = 0; q < NR; ++q)
      acc[q] = fmadd(static_cast<double>(a[static_cast<size_t>(i) * NR + q]),
                     static_cast<double>(b[static_cast<size_t>(i) * NR + q]), acc[q]);
  }
#pragma unroll
  for (int q = 0; q < NR; ++q) {
    acc[q] = group_sum<64>(acc[q]);
    if ((threadIdx.x & 63) == 0) lds[(threadIdx.x >> 6) * NR + q] = acc[q];
  }
  __syncthreads();
  if (threadIdx.x < NR) {
    const int q = threadIdx.x;
    partial[static_cast<size_t>(c) * NR + q] = ((lds[q] + lds[NR + q]) + lds[2 * NR + q]) + lds[3 * NR + q];
  }
}

// Output (segment s, rhs q) = sum of partial[c * nr + q] over the chunks c of s,
// workgroup per output, fixed assignment and tree; then op(s, q, sum).
template <class Op>
__global__ __launch_bounds__(256) void seg_finish_kernel(const double* __restrict__ partial,
                                                         const int32_t* __restrict__ seg_ptr, int nr, Op op) {
  __shared__ double lds[4];
  const int sg = blockIdx.x / nr, q = blockIdx.x % nr;
  double v = 0.0;
  for (int c = seg_ptr[sg] + threadIdx.x; c < seg_ptr[sg + 1]; c += 256) v += partial[static_cast<size_t>(c) * nr + q];
  const double s = block_sum_256(v, lds);
  if (threadIdx.x == 0) op(sg, q, s);
}

// Lanczos scalars of segment s: which < 0 -> tmp[0] = sqrt(v); else beta[which] = sqrt(v)
struct OpLzSqrt {
  LevelScalars* sc;
  int which;
  __device__ void operator()(int s, int, double v) const {
    const double r = sqrt(v > 0.0 ? v : 0.0);
    if (which < 0) sc[s].tmp[0] = r; else sc[s].beta[which] = r;
  }
};
struct OpLzAlpha {
  LevelScalars* sc;
  int step;
  __device__ void operator()(int s, int, double v) const { sc[s].alpha[step] = v; }
};

// ---------------------------------------------------------------------------
// Block-diagonal inverse (point-block Jacobi, paper §4.1)
// ---------------------------------------------------------------------------
template <int BS, class TM, class TD>
__global__ __launch_bounds__(256) void dinv_kernel(int nbr, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                            const TM* __restrict__ val, TD* __restrict__ dinv, int32_t* __restrict__ diag_idx,
                            int* flag) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nbr) return;
  // the diagonal block: binary search in the row's ascending column indices
  int kd = -1;
  for (int lo = rp[r], hi = rp[r + 1]; lo < hi;) {
    const int mid = (lo + hi) >> 1;
    const int c = ci[mid];
    if (c == r) { kd = mid; break; }
    if (c < r) lo = mid + 1; else hi = mid;
  }
  diag_idx[r] = kd;
  double a[BS][2 * BS];
#pragma unroll
  for (int i = 0; i < BS; ++i) {
#pragma unroll
    for (int j = 0; j < BS; ++j) {
      a[i][j] = kd >= 0 ? ld<double>(val + static_cast<size_t>(kd) * BS * BS + i * BS + j) : 0.0;
      a[i][BS + j] = (i == j) ? 1.0 : 0.0;
    }
  }
  // Gauss-Jordan with partial pivoting, fully unrolled: the pivot row is exchanged with
  // row c by selects, so every index is a compile-time constant and the array stays in
  // registers (indexing it by the run-time pivot put it in scratch memory)
  bool ok = kd >= 0;
#pragma unroll
  for (int c = 0; c < BS; ++c) {
    int p = c;
    double best = fabs(a[c][c]);
#pragma unroll
    for (int i = c + 1; i < BS; ++i)
      if (fabs(a[i][c]) > best) { best = fabs(a[i][c]); p = i; }
    ok = ok && best > 0.0;
#pragma unroll
    for (int i = c + 1; i < BS; ++i) {
      const bool sw = i == p;
#pragma unroll
      for (int j = 0; j < 2 * BS; ++j) {
        const double t = a[c][j];
        a[c][j] = sw ? a[i][j] : t;
        a[i][j] = sw ? t : a[i][j];
      }
    }
    const double inv = ok ? 1.0 / a[c][c] : 0.0;
#pragma unroll
    for (int j = 0; j < 2 * BS; ++j) a[c][j] *= inv;
#pragma unroll
    for (int i = 0; i < BS; ++i) {
      if (i == c) continue;
      const double f = a[i][c];
#pragma unroll
      for (int j = 0; j < 2 * BS; ++j) a[i][j] -= f * a[c][j];
    }
  }
  if (!ok) atomicExch(flag, 1);
  TD* o = dinv + static_cast<size_t>(r) * BS * BS;
  for (int i = 0; i < BS; ++i)
    for (int j = 0; j < BS; ++j) o[i * BS + j] = static_cast<TD>(ok ? a[i][BS + j] : (i == j ? 1.0 : 0.0));
}

// ---------------------------------------------------------------------------
// Lanczos (D inner product on D^-1 A), one recurrence per active segment.
// sc points at this level's first LevelScalars; segment s uses sc[s].
// ---------------------------------------------------------------------------

// v from splitmix64 of the instance-local scalar index, Dv = diag-block(A) v
template <int BS, class TM, class TV>
__global__ void lanczos_start_kernel(int nbr, const int32_t* __restrict__ off, int nseg, uint64_t seed,
                                     const TM* __restrict__ val, const int32_t* __restrict__ diag_idx,
                                     TV* __restrict__ v, TV* __restrict__ Dv) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nbr) return;
  const int sg = seg_of(off, nseg, r);
  const int64_t local = static_cast<int64_t>(r - off[sg]) * BS;
  double vv[BS];
  for (int j = 0; j < BS; ++j) {
    const uint64_t z = splitmix64(seed ^ static_cast<uint64_t>(local + j));
    vv[j] = static_cast<double>(static_cast<TV>(2.0 * (static_cast<double>(z >> 11) * 0x1.0p-53) - 1.0));
    v[static_cast<size_t>(r) * BS + j] = static_cast<TV>(vv[j]);
  }
  const int kd = diag_idx[r];
  for (int i = 0; i < BS; ++i) {
    double sv = 0.0;
    if (kd >= 0)
      for (int j = 0; j < BS; ++j) sv += ld<double>(val + static_cast<size_t>(kd) * BS * BS + i * BS + j) * vv[j];
    Dv[static_cast<size_t>(r) * BS + i] = static_cast<TV>(sv);
  }
}

// (ao, bo) = (a, b) / s_seg with s_seg = sc[seg].tmp[0] (start) or sc[seg].beta[step]
template <int BS, class TV>
__global__ void lanczos_scale_kernel(int nbr, const int32_t* __restrict__ off, int nseg,
                                     const LevelScalars* __restrict__ sc, int which, const TV* __restrict__ a,
                                     const TV* __restrict__ b, TV* __restrict__ ao, TV* __restrict__ bo) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nbr) return;
  const int sg = seg_of(off, nseg, r);
  double s = which < 0 ? sc[sg].tmp[0] : sc[sg].beta[which];
  if (!(s > 0.0)) s = 1.0;
  const double inv = 1.0 / s;
  for (int j = 0; j < BS; ++j) {
    const size_t o = static_cast<size_t>(r) * BS + j;
    ao[o] = static_cast<TV>(static_cast<double>(a[o]) * inv);
    bo[o] = static_cast<TV>(static_cast<double>(b[o]) * inv);
  }
}

// wy -= alpha_seg * y ; wu = Dinv wy
template <int BS, class TV>
__global__ void lanczos_orth_kernel(int nbr, const int32_t* __restrict__ off, int nseg,
                                    const LevelScalars* __restrict__ sc, int step, const TV* __restrict__ y,
                                    TV* __restrict__ wy, const TV* __restrict__ dinv, TV* __restrict__ wu) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nbr) return;
  const double al = sc[seg_of(off, nseg, r)].alpha[step];
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
    wu[static_cast<size_t>(r) * BS + i] = static_cast<TV>(z);
  }
}

// SpMV epilogue: wy = A u - beta_{step-1, seg} * y_prev (no previous vector on step 0);
// one right-hand side, BR <= G: lane i < BR owns output i
template <class TV, class TA>
struct EpiLanczos {
  static constexpr bool kReduce = false;
  const TV* y_prev;
  TV* wy;
  const LevelScalars* sc;
  const int32_t* off;
  int nseg;
  int step;
  double* partial = nullptr;
  template <int BR, int NR, int G>
  __device__ __forceinline__ RowVals<double, 2> prefetch(bool active, int row) const {
    static_assert(lane_owned<BR * NR, G>(), "Lanczos epilogue expects BR * NR <= G");
    RowVals<double, 2> p;
    p.v[0] = 0.0;
    p.v[1] = 0.0;
    const int lane = static_cast<int>(threadIdx.x) % G;
    if (active && step > 0 && lane < BR * NR) {
      p.v[1] = sc[seg_of(off, nseg, row)].beta[step - 1];
      p.v[0] = static_cast<double>(y_prev[static_cast<size_t>(row) * (BR * NR) + lane]);
    }
    return p;
  }
  template <int BR, int NR, int G>
  __device__ __forceinline__ double apply(bool active, int row, int lane, const TA (&s)[BR * NR],
                                          const RowVals<double, 2>& pre) const {
    if (!active || lane >= BR * NR) return 0.0;
    wy[static_cast<size_t>(row) * (BR * NR) + lane] =
        static_cast<TV>(static_cast<double>(pick<BR * NR>(s, lane)) - pre.v[1] * pre.v[0]);
    return 0.0;
  }
};

// Largest eigenvalue of each segment's tridiagonal T_k by Sturm bisection, then the
// Chebyshev coefficients (Saad, Alg. 12.1) for [lo*lam, hi*lam].  One thread per segment.
__global__ void lanczos_finish_kernel(LevelScalars* sc, int nseg, int k, const double* user_lam, double lo,
                                      double hi, int degree) {
  const int sg = blockIdx.x * blockDim.x + threadIdx.x;
  if (sg >= nseg) return;
  LevelScalars* S = sc + sg;
  double lam;
  if (user_lam != nullptr) {
    lam = user_lam[sg];
  } else {
    int m = k;
    for (int j = 0; j < k - 1; ++j)
      if (!(S->beta[j] > 0.0)) { m = j + 1; break; }
    double gl = 1e300, gh = -1e300;
    for (int i = 0; i < m; ++i) {
      const double o = (i > 0 ? fabs(S->beta[i - 1]) : 0.0) + (i < m - 1 ? fabs(S->beta[i]) : 0.0);
      gl = fmin(gl, S->alpha[i] - o);
      gh = fmax(gh, S->alpha[i] + o);
    }
    double a = gl, b = gh;
    for (int it = 0; it < 200; ++it) {
      const double x = 0.5 * (a + b);
      if (x <= a || x >= b) break;
      int cnt = 0;
      double q = S->alpha[0] - x;
      if (q < 0) cnt++;
      for (int i = 1; i < m; ++i) {
        const double qq = (q != 0.0) ? q : 1e-300;
        q = S->alpha[i] - x - S->beta[i - 1] * S->beta[i - 1] / qq;
        if (q < 0) cnt++;
      }
      if (cnt == m) b = x; else a = x;
    }
    lam = 0.5 * (a + b);
  }
  S->lam = lam;
  const double ea = lo * lam, eb = hi * lam;
  const double theta = 0.5 * (eb + ea), delta = 0.5 * (eb - ea);
  const double sigma = theta / delta;
  double rho = 1.0 / sigma;
  S->coef[0] = 1.0 / theta;
  for (int t = 1; t < degree; ++t) {
    const double rho1 = 1.0 / (2.0 * sigma - rho);
    S->coef[1 + 2 * (t - 1)] = rho1 * rho;
    S->coef[2 + 2 * (t - 1)] = 2.0 * rho1 / delta;
    rho = rho1;
  }
  for (int t = 0; t < 2 * degree - 1; ++t) S->coef_f[t] = static_cast<float>(S->coef[t]);
}

// ---------------------------------------------------------------------------
// Chebyshev / point-block Jacobi (paper §4.1 pbjacobi inside Saad's Chebyshev)
// ---------------------------------------------------------------------------

// d = Dinv f / theta_seg (zero-guess start), NR right-hand sides; row_seg (NULL for
// one segment) gives the segment of each row
template <int BS, int NR, class TV>
__global__ void cheb0_kernel(int nbr, const uint16_t* __restrict__ row_seg, const LevelScalars* __restrict__ sc,
                             const TV* __restrict__ f, const TV* __restrict__ dinv, TV* __restrict__ out) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nbr) return;
  const TV it = cheb_coef<TV>(sc[row_seg ? row_seg[r] : 0], 0);
  TV fv[BS * NR];
  for (int t = 0; t < BS * NR; ++t) fv[t] = f[static_cast<size_t>(r) * BS * NR + t];
  const TV* D = dinv + static_cast<size_t>(r) * BS * BS;
  for (int i = 0; i < BS; ++i)
    for (int q = 0; q < NR; ++q) {
      TV z = 0;
      for (int j = 0; j < BS; ++j) z = fmadd(D[i * BS + j], fv[j * NR + q], z);
      out[static_cast<size_t>(r) * BS * NR + i * NR + q] = z * it;
    }
}

enum SmoothMode { M_RESID = 0, M_INITX = 1, M_STEP = 2 };

// s = A * (gathered vector); per-row Chebyshev coefficients from the row's segment.
//   RESID : r_out = f - s
//   INITX : r = f - s ; d = Dinv r / theta ; x_out = x_in + d   (writes r, d, x_out)
//   STEP  : r = f - s (f = current r) ; d' = c1 d_in + c2 Dinv r ; x_out = x_in + d'
// One right-hand side: lane i < BR owns output i; it loads f_i, d_i, x_i, row i of
// Dinv and the two coefficients before the product (their latency then hides behind
// the block loads), and the residual entries reach the other owners by shuffles.
// Eight right-hand sides: lane q < 8 owns column q of the row (all BR entries), so
// D^-1 r stays inside the lane; its operands are loaded after the product.
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
  const LevelScalars* sc;
  const uint16_t* row_seg;  // segment of each row, NULL for one segment
  int step;
  double* partial = nullptr;

  template <int BR, int NR, int G>
  static constexpr int pre_len() { return 3 + BR; }

  __device__ __forceinline__ const LevelScalars& scal(int row) const { return sc[row_seg ? row_seg[row] : 0]; }

  // own-row operands of one right-hand side, all in the arithmetic type (the
  // coefficients come pre-rounded), so nothing has to be converted, and waited for,
  // before the product
  template <int BR, int NR, int G>
  struct Pre {
    RowVals<TA, 3 + BR> a;
    TA c1, c2;
  };

  // The loads are unconditional (lanes >= BR and rows past the end read valid
  // addresses of the same row / row 0 and their values are never stored), so no
  // branch separates them from the product's loads.
  template <int BR, int NR, int G>
  __device__ __forceinline__ Pre<BR, NR, G> prefetch(bool active, int row) const {
    static_assert(NR == 1 && lane_owned<BR, G>(), "one right-hand side with BR <= G");
    Pre<BR, NR, G> p;
#pragma unroll
    for (int t = 0; t < 3 + BR; ++t) p.a.v[t] = TA(0);
    p.c1 = TA(0);
    p.c2 = TA(0);
    const int lane = min(static_cast<int>(threadIdx.x) % G, BR - 1);
    const int rr = active ? row : 0;
    const size_t o = static_cast<size_t>(rr) * BR + lane;
    p.a.v[0] = ld<TA>(f + o);
    if (MODE == M_STEP) p.a.v[1] = ld<TA>(d_in + o);
    if (MODE != M_RESID) {
      p.a.v[2] = ld<TA>(x_in + o);
      const TV* D = dinv + static_cast<size_t>(rr) * (BR * BR) + lane * BR;
#pragma unroll
      for (int j = 0; j < BR; ++j) p.a.v[3 + j] = ld<TA>(D + j);
      const LevelScalars& S = scal(rr);
      if (MODE == M_INITX) {
        p.c2 = cheb_coef<TA>(S, 0);
      } else {
        p.c1 = cheb_coef<TA>(S, 1 + 2 * step);
        p.c2 = cheb_coef<TA>(S, 2 + 2 * step);
      }
    }
    return p;
  }

  template <int BR, int NR, int G>
  __device__ __forceinline__ double apply(bool active, int row, int lane, const TA (&s)[BR * NR],
                                          const Pre<BR, NR, G>& pre) const {
    if (!active) return 0.0;
    // every lane of the group takes part in the shuffles; lanes >= BR carry zeros
    const TA r = pre.a.v[0] - pick<BR>(s, lane < BR ? lane : 0);
    const size_t o = static_cast<size_t>(row) * BR + lane;
    if (MODE == M_RESID) {
      if (lane < BR) r_out[o] = static_cast<TV>(r);
      return 0.0;
    }
    TA z = TA(0);
#pragma unroll
    for (int j = 0; j < BR; ++j) z = fmadd(pre.a.v[3 + j], __shfl(r, j, G), z);
    TA dn = pre.c2 * z;
    if (MODE == M_STEP) dn = fmadd(pre.c1, pre.a.v[1], dn);
    if (lane < BR) {
      x_out[o] = static_cast<TV>(pre.a.v[2] + dn);
      if (r_out) r_out[o] = static_cast<TV>(r);
      if (d_out) d_out[o] = static_cast<TV>(dn);
    }
    return 0.0;
  }

  template <int BR, int G>
  __device__ __forceinline__ void apply8(bool active, int row, int lane, const TA (&s)[BR]) const {
    if (!active || lane >= 8) return;
    const size_t base = static_cast<size_t>(row) * (BR * 8) + lane;
    TA r[BR];
#pragma unroll
    for (int i = 0; i < BR; ++i) r[i] = ld<TA>(f + base + i * 8) - s[i];
    if (MODE == M_RESID) {
#pragma unroll
      for (int i = 0; i < BR; ++i) r_out[base + i * 8] = static_cast<TV>(r[i]);
      return;
    }
    const LevelScalars& S = scal(row);
    const TA c1 = MODE == M_STEP ? cheb_coef<TA>(S, 1 + 2 * step) : TA(0);
    const TA c2 = MODE == M_STEP ? cheb_coef<TA>(S, 2 + 2 * step) : cheb_coef<TA>(S, 0);
    const TV* D = dinv + static_cast<size_t>(row) * (BR * BR);
#pragma unroll
    for (int i = 0; i < BR; ++i) {
      TA z = TA(0);
#pragma unroll
      for (int j = 0; j < BR; ++j) z = fmadd(ld<TA>(D + i * BR + j), r[j], z);
      const size_t o = base + i * 8;
      TA dn = c2 * z;
      if (MODE == M_STEP) dn = fmadd(c1, ld<TA>(d_in + o), dn);
      x_out[o] = static_cast<TV>(ld<TA>(x_in + o) + dn);
      if (r_out) r_out[o] = static_cast<TV>(r[i]);
      if (d_out) d_out[o] = static_cast<TV>(dn);
    }
  }
};

// ---------------------------------------------------------------------------
// Prolongator smoothing (cold setup, paper §2.2) with the weight omega of the row's
// segment (omega_scale / lambda_hat, or a learned weight):
//   P_ib = [agg(i) == b] P~_i - omega Dinv_i sum_{j in A_i, agg(j) == b} A_ij P~_j
// ---------------------------------------------------------------------------
template <int BS, int NC>
__global__ void smooth_p_kernel(int nbr, const int32_t* __restrict__ a_rp, const int32_t* __restrict__ a_ci,
                                const double* __restrict__ a_v, const int32_t* __restrict__ agg,
                                const double* __restrict__ pt, const double* __restrict__ dinv,
                                const int32_t* __restrict__ off, int nseg, const double* __restrict__ omega_seg,
                                const int32_t* __restrict__ p_rp, const int32_t* __restrict__ p_ci,
                                double* __restrict__ p_v) {
  const int64_t gidx = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
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
  const double omega = omega_seg[seg_of(off, nseg, i)];
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
// Dense coarse solves (FP64) of all terminal segments of a level at once:
// expansion, blocked Cholesky, inverse of the factor.  Segment t (blockIdx.y) owns
// an n_t x n_t row-major matrix at mats + mat_off[t]; tiles of kT x kT, and tiles
// that stick out of the matrix act as identity-padded.
// ---------------------------------------------------------------------------
constexpr int kT = 32;

// block rows [row0_t, row0_t + nrows_t) of the level matrix, columns shifted by row0_t
template <class TM>
__global__ void expand_dense_kernel(const int32_t* __restrict__ seg_row0, const int32_t* __restrict__ seg_nrows,
                                    const int64_t* __restrict__ mat_off, int bs, const int32_t* __restrict__ rp,
                                    const int32_t* __restrict__ ci, const TM* __restrict__ val,
                                    double* __restrict__ mats) {
  const int t = blockIdx.y;
  const int r = blockIdx.x;
  const int nr = seg_nrows[t], r0 = seg_row0[t];
  if (r >= nr) return;
  const int n = nr * bs;
  double* M = mats + mat_off[t];
  for (int k = rp[r0 + r]; k < rp[r0 + r + 1]; ++k) {
    const int c = ci[k] - r0;
    if (c < 0 || c >= nr) continue;
    for (int e = threadIdx.x; e < bs * bs; e += blockDim.x) {
      const int i = e / bs, j = e % bs;
      M[static_cast<size_t>(r * bs + i) * n + c * bs + j] = ld<double>(val + static_cast<size_t>(k) * bs * bs + e);
    }
  }
}

__device__ __forceinline__ double mat_at(const double* M, int n, int i, int j) {
  if (i < n && j < n) return M[static_cast<size_t>(i) * n + j];
  return (i == j) ? 1.0 : 0.0;
}

__device__ inline void factor_diag_tile(const double* M, int n, int k, double (*D)[kT + 1], int* flag) {
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

__device__ __forceinline__ int tiles_of(int n) { return (n + kT - 1) / kT; }

// Panel k: block 0 writes L_kk; block b > 0 writes L_{k+b,k} = A_{k+b,k} L_kk^-T.
__global__ __launch_bounds__(256) void chol_panel_kernel(double* __restrict__ mats, const int64_t* __restrict__ mat_off,
                                                         const int32_t* __restrict__ ndof, int k, int* flag) {
  __shared__ double D[kT][kT + 1];
  __shared__ double X[kT][kT + 1];
  const int n = ndof[blockIdx.y];
  const int nt = tiles_of(n);
  if (k >= nt || k + static_cast<int>(blockIdx.x) >= nt) return;  // uniform over the block
  double* M = mats + mat_off[blockIdx.y];
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
  if (threadIdx.x < kT) {  // row r of X: x_j = (a_j - sum_{m<j} x_m L_jm) / L_jj
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

// Trailing update after panel k: A_IJ -= L_Ik L_Jk^T over the lower tiles of the
// trailing part; block x enumerates those tiles row by row.
__global__ __launch_bounds__(256) void chol_update_kernel(double* __restrict__ mats, const int64_t* __restrict__ mat_off,
                                                          const int32_t* __restrict__ ndof, int k) {
  __shared__ double Li[kT][kT + 1];
  __shared__ double Lj[kT][kT + 1];
  const int n = ndof[blockIdx.y];
  const int m = tiles_of(n) - k - 1;
  if (m <= 0 || static_cast<int>(blockIdx.x) >= m * (m + 1) / 2) return;
  double* M = mats + mat_off[blockIdx.y];
  int t = blockIdx.x, I = 0;
  while (t >= I + 1) { t -= I + 1; ++I; }
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

// Column block J of Y = L^-1 by block forward substitution,
//   Y_IJ = L_II^-1 (delta_IJ - sum_{K=J}^{I-1} L_IK Y_KJ),  I = J .. nt-1,
// one workgroup per column block (block x = J), all of Y in one launch: the columns
// are independent, and each workgroup reads back only tiles it wrote itself (visible
// after the block barrier).
__global__ __launch_bounds__(256) void tri_inverse_col_kernel(const double* __restrict__ Ls, double* __restrict__ Ys,
                                                              const int64_t* __restrict__ mat_off,
                                                              const int32_t* __restrict__ ndof) {
  __shared__ double Dd[kT][kT + 1];
  __shared__ double S[kT][kT + 1];
  __shared__ double A[kT][kT + 1];
  __shared__ double Bt[kT][kT + 1];
  const int n = ndof[blockIdx.y];
  const int nt = tiles_of(n);
  const int J = blockIdx.x;
  if (J >= nt) return;  // uniform over the block
  const double* L = Ls + mat_off[blockIdx.y];
  double* Y = Ys + mat_off[blockIdx.y];
  const int cj = J * kT;
  for (int I = J; I < nt; ++I) {
    const int ri = I * kT;
    for (int e = threadIdx.x; e < kT * kT; e += blockDim.x) {
      const int i = e / kT, j = e % kT;
      Dd[i][j] = mat_at(L, n, ri + i, ri + j);
      S[i][j] = (I == J && i == j) ? 1.0 : 0.0;
    }
    __syncthreads();
    // the tiles of step K + 1 are loaded into registers while step K multiplies
    constexpr int kPer = kT * kT / 256;  // elements of a tile per thread
    double na[kPer], nb[kPer];
    auto fetch = [&](int K) {
      const int rk = K * kT;
#pragma unroll
      for (int u = 0; u < kPer; ++u) {
        const int e = static_cast<int>(threadIdx.x) + u * 256;
        const int i = e / kT, j = e % kT;
        na[u] = (ri + i < n && rk + j < n) ? L[static_cast<size_t>(ri + i) * n + rk + j] : 0.0;
        nb[u] = (rk + i < n && cj + j < n) ? Y[static_cast<size_t>(rk + i) * n + cj + j] : 0.0;
      }
    };
    if (J < I) fetch(J);
    for (int K = J; K < I; ++K) {
#pragma unroll
      for (int u = 0; u < kPer; ++u) {
        const int e = static_cast<int>(threadIdx.x) + u * 256;
        A[e / kT][e % kT] = na[u];
        Bt[e / kT][e % kT] = nb[u];
      }
      __syncthreads();
      if (K + 1 < I) fetch(K + 1);
      for (int e = threadIdx.x; e < kT * kT; e += blockDim.x) {
        const int i = e / kT, j = e % kT;
        double sdot = 0.0;
#pragma unroll 8
        for (int q = 0; q < kT; ++q) sdot += A[i][q] * Bt[q][j];
        S[i][j] -= sdot;
      }
      __syncthreads();
    }
    if (threadIdx.x < kT) {  // forward substitution L_II y = s, column j by thread j
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
    __syncthreads();  // this tile is read back (as Y_KJ) by the next block rows
  }
}

// Yt_t = Y_t^T for every segment
__global__ void transpose_dense_kernel(const double* __restrict__ Ys, double* __restrict__ Yts,
                                       const int64_t* __restrict__ mat_off, const int32_t* __restrict__ ndof) {
  const int n = ndof[blockIdx.y];
  const size_t e = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x;
  if (e >= static_cast<size_t>(n) * n) return;
  const int i = static_cast<int>(e / n), j = static_cast<int>(e % n);
  Yts[mat_off[blockIdx.y] + static_cast<size_t>(j) * n + i] = Ys[mat_off[blockIdx.y] + e];
}

// y[seg] = M_seg x[seg] for every terminal segment of a level; one wave per row.
// seg t covers scalar rows [dof_off[t], dof_off[t+1]) of the level vectors (relative
// to dof0), its n x n matrix starts at mat_off[t]; row i uses columns [0, i] (lower)
// or [i, n) (upper).
template <int NR, class TI, class TO>
__global__ __launch_bounds__(256) void dense_tri_batched_kernel(const double* __restrict__ mats,
                                                                const int64_t* __restrict__ mat_off,
                                                                const int32_t* __restrict__ dof_off, int nseg,
                                                                int dof0, int upper, const TI* __restrict__ x,
                                                                TO* __restrict__ y) {
  const int grow = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (grow >= dof_off[nseg]) return;
  const int t = seg_of(dof_off, nseg, grow);
  const int n = dof_off[t + 1] - dof_off[t];
  const int i = grow - dof_off[t];
  const double* Mr = mats + mat_off[t] + static_cast<int64_t>(i) * n;
  const size_t xb = static_cast<size_t>(dof0 + dof_off[t]) * NR;
  const int lo = upper ? i : 0, hi = upper ? n : i + 1;
  double s[NR];
#pragma unroll
  for (int q = 0; q < NR; ++q) s[q] = 0.0;
  for (int k = lo + lane; k < hi; k += 64) {
    const double m = Mr[k];
#pragma unroll
    for (int q = 0; q < NR; ++q) s[q] = fmadd(m, static_cast<double>(x[xb + static_cast<size_t>(k) * NR + q]), s[q]);
  }
#pragma unroll
  for (int q = 0; q < NR; ++q) s[q] = group_sum<64>(s[q]);
  if (lane < NR) {
    double v = 0.0;
#pragma unroll
    for (int q = 0; q < NR; ++q)
      if (q == lane) v = s[q];
    y[xb + static_cast<size_t>(i) * NR + lane] = static_cast<TO>(v);
  }
}

template <class TI, class TO>
__global__ void cast_vec_kernel(size_t n, const TI* __restrict__ a, TO* __restrict__ b) {
  const size_t g = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x;
  if (g < n) b[g] = static_cast<TO>(a[g]);
}

// ---------------------------------------------------------------------------
// Single-system CG kernels (fused path)
// ---------------------------------------------------------------------------
enum { S_RZ = 0, S_PW, S_ALPHA, S_RR, S_BETA, S_BB, S_FLAG, S_COUNT };

struct EpiPcgW {
  static constexpr bool kReduce = true;
  const double* p;
  double* w;
  double* partial;
  // one right-hand side, lane i < BR owns output i
  template <int BR, int NR, int G>
  __device__ __forceinline__ RowVals<double, 1> prefetch(bool active, int row) const {
    static_assert(lane_owned<BR * NR, G>(), "CG epilogue expects BR * NR <= G");
    RowVals<double, 1> pv;
    const int lane = min(static_cast<int>(threadIdx.x) % G, BR * NR - 1);
    pv.v[0] = p[static_cast<size_t>(active ? row : 0) * (BR * NR) + lane];  // unconditional, see EpiSmooth
    return pv;
  }
  template <int BR, int NR, int G>
  __device__ __forceinline__ double apply(bool active, int row, int lane, const double (&s)[BR * NR],
                                          const RowVals<double, 1>& pre) const {
    if (!active || lane >= BR * NR) return 0.0;
    const double v = pick<BR * NR>(s, lane);
    w[static_cast<size_t>(row) * (BR * NR) + lane] = v;
    return pre.v[0] * v;
  }
};

// x += alpha p, r -= alpha w, partial sums of r.r; with r32 set, also the FP32 copy of r
// that an FP32 V-cycle takes as input (rounded to nearest)
__global__ __launch_bounds__(256) void pcg_update_kernel(size_t n, const double* __restrict__ sc,
                                                         const double* __restrict__ p, const double* __restrict__ w,
                                                         double* __restrict__ x, double* __restrict__ r,
                                                         double* __restrict__ partial, float* __restrict__ r32) {
  __shared__ double lds[4];
  double acc = 0.0;
  const double a = sc[S_ALPHA];
  for (size_t g = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x; g < n;
       g += static_cast<size_t>(gridDim.x) * blockDim.x) {
    x[g] = fmadd(a, p[g], x[g]);
    const double rv = fmadd(-a, w[g], r[g]);
    r[g] = rv;
    if (r32) r32[g] = static_cast<float>(rv);
    acc = fmadd(rv, rv, acc);
  }
  const double t = block_sum_256(acc, lds);
  if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

// partial sums of a.b; b may be the FP32 output of an FP32 V-cycle (widened exactly)
template <class TB>
__global__ __launch_bounds__(256) void dot_kernel(size_t n, const double* __restrict__ a, const TB* __restrict__ b,
                                                  double* __restrict__ partial) {
  __shared__ double lds[4];
  double acc = 0.0;
  for (size_t g = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x; g < n;
       g += static_cast<size_t>(gridDim.x) * blockDim.x)
    acc = fmadd(a[g], static_cast<double>(b[g]), acc);
  const double t = block_sum_256(acc, lds);
  if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

template <class TZ>
__global__ void pcg_p_kernel(size_t n, const double* __restrict__ sc, int use_beta, const TZ* __restrict__ z,
                             double* __restrict__ p) {
  const size_t g = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x;
  if (g >= n) return;
  const double zv = static_cast<double>(z[g]);
  p[g] = use_beta ? fmadd(sc[S_BETA], p[g], zv) : zv;
}

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
// Batched CG: one independent recurrence per (instance, right-hand side).
// Scalars are stored [field][seg * nr + q]; a converged system gets alpha = 0 and
// keeps its x and r.
// ---------------------------------------------------------------------------
enum { B_RZ = 0, B_PW, B_ALPHA, B_RR, B_BETA, B_BB, B_DONE, B_ITS, B_FIELDS };

// Field f of system k = (segment, rhs) lives at bs[f * stride + k].
__device__ __forceinline__ double& bf(double* bs, int stride, int f, int k) { return bs[f * stride + k]; }

// bb = b.b ; start the system (done = 1 when b = 0, = 3 when maxit = 0)
struct OpBInit {
  double* bs;
  int stride, nr, maxit;
  __device__ void operator()(int s, int q, double v) const {
    const int k = s * nr + q;
    bf(bs, stride, B_BB, k) = v;
    bf(bs, stride, B_RR, k) = v;
    bf(bs, stride, B_ITS, k) = 0.0;
    bf(bs, stride, B_ALPHA, k) = 0.0;
    bf(bs, stride, B_BETA, k) = 0.0;
    bf(bs, stride, B_DONE, k) = !(v > 0.0) ? 1.0 : (maxit <= 0 ? 3.0 : 0.0);
  }
};
struct OpBRz0 {
  double* bs;
  int stride, nr;
  __device__ void operator()(int s, int q, double v) const { bf(bs, stride, B_RZ, s * nr + q) = v; }
};
// pw = p.w ; alpha = rz / pw for running systems (breakdown: done = 2)
struct OpBAlpha {
  double* bs;
  int stride, nr;
  __device__ void operator()(int s, int q, double v) const {
    const int k = s * nr + q;
    bf(bs, stride, B_PW, k) = v;
    double a = 0.0;
    if (bf(bs, stride, B_DONE, k) == 0.0) {
      if (!(v > 0.0)) bf(bs, stride, B_DONE, k) = 2.0;
      else a = bf(bs, stride, B_RZ, k) / v;
    }
    bf(bs, stride, B_ALPHA, k) = a;
  }
};
// rr = r.r ; count the update, stop at ||r|| <= rtol ||b|| (done = 1) or maxit (done = 3)
struct OpBRr {
  double* bs;
  int stride, nr, maxit;
  double rtol;
  __device__ void operator()(int s, int q, double v) const {
    const int k = s * nr + q;
    if (bf(bs, stride, B_DONE, k) != 0.0) return;
    bf(bs, stride, B_RR, k) = v;
    const double its = bf(bs, stride, B_ITS, k) + 1.0;
    bf(bs, stride, B_ITS, k) = its;
    if (sqrt(v) <= rtol * sqrt(bf(bs, stride, B_BB, k))) bf(bs, stride, B_DONE, k) = 1.0;
    else if (its >= maxit) bf(bs, stride, B_DONE, k) = 3.0;
  }
};
// rz' = r.z ; beta = rz' / rz for running systems
struct OpBBeta {
  double* bs;
  int stride, nr;
  __device__ void operator()(int s, int q, double v) const {
    const int k = s * nr + q;
    double b = 0.0;
    if (bf(bs, stride, B_DONE, k) == 0.0) {
      b = v / bf(bs, stride, B_RZ, k);
      bf(bs, stride, B_RZ, k) = v;
    }
    bf(bs, stride, B_BETA, k) = b;
  }
};

// stat[0] = systems still running, stat[1] = systems that broke down
__global__ void bpcg_status_kernel(const double* __restrict__ bs, int stride, int nsys, int32_t* __restrict__ stat) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  int run = 0, brk = 0;
  for (int k = 0; k < nsys; ++k) {
    const double d = bs[B_DONE * stride + k];
    run += d == 0.0;
    brk += d == 2.0;
  }
  stat[0] = run;
  stat[1] = brk;
}

// r = b, x = 0
__global__ void bpcg_init_kernel(size_t n, const double* __restrict__ b, double* __restrict__ x,
                                 double* __restrict__ r) {
  const size_t g = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x;
  if (g >= n) return;
  r[g] = b[g];
  x[g] = 0.0;
}

// x += alpha p ; r -= alpha w   (alpha of the element's system; systems with alpha = 0
// are left untouched, so a stopped system keeps its x and r exactly)
// x += alpha p, r -= alpha w per system (alpha = 0: frozen, untouched); with r32 set,
// also the FP32 copy of r that an FP32 V-cycle takes as input
__global__ void bpcg_axpy_kernel(size_t nrow, int nr, const int32_t* __restrict__ off, int nseg,
                                 const double* __restrict__ bs, int stride, const double* __restrict__ p,
                                 const double* __restrict__ w, double* __restrict__ x, double* __restrict__ r,
                                 float* __restrict__ r32) {
  const size_t g = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x;
  if (g >= nrow * nr) return;
  const int row = static_cast<int>(g / nr), q = static_cast<int>(g % nr);
  const int sg = nseg > 1 ? seg_of(off, nseg, row) : 0;
  const double a = bs[B_ALPHA * stride + sg * nr + q];
  if (a == 0.0) return;
  x[g] = fmadd(a, p[g], x[g]);
  const double rv = fmadd(-a, w[g], r[g]);
  r[g] = rv;
  if (r32) r32[g] = static_cast<float>(rv);
}

// p = z + beta p  (p = z on the first step or when beta = 0)
template <class TZ>
__global__ void bpcg_p_kernel(size_t nrow, int nr, const int32_t* __restrict__ off, int nseg,
                              const double* __restrict__ bs, int stride, int use_beta, const TZ* __restrict__ z,
                              double* __restrict__ p) {
  const size_t g = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x;
  if (g >= nrow * nr) return;
  double v = static_cast<double>(z[g]);
  if (use_beta) {
    const int row = static_cast<int>(g / nr), q = static_cast<int>(g % nr);
    const int sg = nseg > 1 ? seg_of(off, nseg, row) : 0;
    const double b = bs[B_BETA * stride + sg * nr + q];
    if (b != 0.0) v = fmadd(b, p[g], v);
  }
  p[g] = v;
}

// ---------------------------------------------------------------------------
// Learned eigenbound support: level features, reference Lanczos with full
// reorthogonalisation (the judge), smoother growth test
// ---------------------------------------------------------------------------
constexpr int kFeatStats = 9;  // sum g, sum g^2, max g, sum h, max h, max d, min d, sum nb, max nb

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
}
__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmin(v, __shfl_xor(v, off, 64));
  return v;
}

// Per chunk of block rows: g_i = max scalar row of |D_i^-1 [A_i1 .. A_in]| summed,
// h_i = sum_{j != i} ||D_i^-1 A_ij||_F, d_i = ||A_ii||_F, nb_i = blocks in the row;
// partial[c][kFeatStats] holds the chunk's sums / maxima / minimum.
template <int BS, class TM, class TD>
__global__ __launch_bounds__(256) void feature_stats_kernel(const int32_t* __restrict__ rp,
                                                            const int32_t* __restrict__ ci,
                                                            const TM* __restrict__ val, const TD* __restrict__ dinv,
                                                            const int32_t* __restrict__ lo,
                                                            const int32_t* __restrict__ hi,
                                                            double* __restrict__ partial) {
  __shared__ double lsum[5][4];
  __shared__ double lext[4][4];
  const int c = blockIdx.x;
  const int r0 = lo[c] / BS, r1 = hi[c] / BS;
  double sg = 0.0, sg2 = 0.0, mg = 0.0, sh = 0.0, mh = 0.0, md = 0.0, mnd = 1e300, snb = 0.0, mnb = 0.0;
  for (int r = r0 + static_cast<int>(threadIdx.x); r < r1; r += 256) {
    double D[BS * BS];
    for (int t = 0; t < BS * BS; ++t) D[t] = static_cast<double>(dinv[static_cast<size_t>(r) * BS * BS + t]);
    double rows[BS];
    for (int i = 0; i < BS; ++i) rows[i] = 0.0;
    double h = 0.0, d = 0.0;
    for (int k = rp[r]; k < rp[r + 1]; ++k) {
      const TM* a = val + static_cast<size_t>(k) * BS * BS;
      double fro = 0.0;
      for (int i = 0; i < BS; ++i)
        for (int j = 0; j < BS; ++j) {
          double m = 0.0;
          for (int q = 0; q < BS; ++q) m += D[i * BS + q] * ld<double>(a + q * BS + j);
          rows[i] += fabs(m);
          fro += m * m;
        }
      if (ci[k] == r) {
        double dd = 0.0;
        for (int t = 0; t < BS * BS; ++t) dd += ld<double>(a + t) * ld<double>(a + t);
        d = sqrt(dd);
      } else {
        h += sqrt(fro);
      }
    }
    double g = rows[0];
    for (int i = 1; i < BS; ++i) g = fmax(g, rows[i]);
    const double nb = static_cast<double>(rp[r + 1] - rp[r]);
    sg += g;
    sg2 += g * g;
    mg = fmax(mg, g);
    sh += h;
    mh = fmax(mh, h);
    md = fmax(md, d);
    mnd = fmin(mnd, d);
    snb += nb;
    mnb = fmax(mnb, nb);
  }
  const double t0 = block_sum_256(sg, lsum[0]);
  const double t1 = block_sum_256(sg2, lsum[1]);
  const double t3 = block_sum_256(sh, lsum[2]);
  const double t7 = block_sum_256(snb, lsum[3]);
  const int w = threadIdx.x >> 6;
  mg = wave_max(mg);
  mh = wave_max(mh);
  md = wave_max(md);
  mnd = wave_min(mnd);
  mnb = wave_max(mnb);
  if ((threadIdx.x & 63) == 0) {
    lext[0][w] = mg;
    lext[1][w] = mh;
    lext[2][w] = md;
    lext[3][w] = mnd;
    lsum[4][w] = mnb;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double* o = partial + static_cast<size_t>(c) * kFeatStats;
    o[0] = t0;
    o[1] = t1;
    o[2] = fmax(fmax(lext[0][0], lext[0][1]), fmax(lext[0][2], lext[0][3]));
    o[3] = t3;
    o[4] = fmax(fmax(lext[1][0], lext[1][1]), fmax(lext[1][2], lext[1][3]));
    o[5] = fmax(fmax(lext[2][0], lext[2][1]), fmax(lext[2][2], lext[2][3]));
    o[6] = fmin(fmin(lext[3][0], lext[3][1]), fmin(lext[3][2], lext[3][3]));
    o[7] = t7;
    o[8] = fmax(fmax(lsum[4][0], lsum[4][1]), fmax(lsum[4][2], lsum[4][3]));
  }
}

// Features of segment s (one thread each) from its chunks, in chunk order.
__global__ void feature_finish_kernel(const double* __restrict__ partial, const int32_t* __restrict__ seg_ptr,
                                      const int32_t* __restrict__ row_off, int nseg, int bs, int level,
                                      float* __restrict__ feat) {
  const int sg = blockIdx.x * blockDim.x + threadIdx.x;
  if (sg >= nseg) return;
  double st[kFeatStats] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 1e300, 0.0, 0.0};
  for (int c = seg_ptr[sg]; c < seg_ptr[sg + 1]; ++c) {
    const double* p = partial + static_cast<size_t>(c) * kFeatStats;
    st[0] += p[0];
    st[1] += p[1];
    st[2] = fmax(st[2], p[2]);
    st[3] += p[3];
    st[4] = fmax(st[4], p[4]);
    st[5] = fmax(st[5], p[5]);
    st[6] = fmin(st[6], p[6]);
    st[7] += p[7];
    st[8] = fmax(st[8], p[8]);
  }
  const double nr = static_cast<double>(row_off[sg + 1] - row_off[sg]);
  float* f = feat + static_cast<size_t>(sg) * 12;
  const double mean_g = st[0] / nr;
  f[0] = static_cast<float>(log(st[2]));
  f[1] = static_cast<float>(log(mean_g));
  f[2] = static_cast<float>(log(sqrt(st[1] / nr)));
  f[3] = static_cast<float>(log1p(st[4]));
  f[4] = static_cast<float>(log1p(st[3] / nr));
  f[5] = static_cast<float>(log(st[5] / st[6]));
  f[6] = static_cast<float>(st[7] / nr);
  f[7] = static_cast<float>(st[8]);
  f[8] = static_cast<float>(log(nr * bs));
  f[9] = static_cast<float>(level);
  f[10] = static_cast<float>(bs / 6.0);
  f[11] = static_cast<float>(log1p(st[3] / nr) - log(mean_g));
}

// x = (f - mean) / std per feature (model statistics after the parameters)
__global__ void feature_normalize_kernel(int n, const float* __restrict__ feat, const float* __restrict__ stats,
                                         float* __restrict__ x) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * 12) return;
  const int j = e % 12;
  x[e] = (feat[e] - stats[j]) / stats[12 + j];
}

// network outputs -> lambda = exp(y0 sd0 + mu0), omega = y1 sd1 + mu1
__global__ void predict_finish_kernel(int n, const float* __restrict__ y, const float* __restrict__ tstats,
                                      double* __restrict__ lam, double* __restrict__ omega) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  lam[i] = exp(static_cast<double>(y[2 * i]) * tstats[2] + tstats[0]);
  omega[i] = static_cast<double>(y[2 * i + 1]) * tstats[3] + tstats[1];
}

// wy -= alpha_seg y + beta_seg y_prev (beta part only when y_prev != NULL)
template <int BS>
__global__ void judge_orth_kernel(int nbr, const int32_t* __restrict__ off, int nseg,
                                  const LevelScalars* __restrict__ sc, int step, const double* __restrict__ y,
                                  const double* __restrict__ y_prev, double* __restrict__ wy) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nbr) return;
  const LevelScalars& S = sc[seg_of(off, nseg, r)];
  const double al = S.alpha[step];
  const double be = y_prev ? S.beta[step - 1] : 0.0;
  for (int j = 0; j < BS; ++j) {
    const size_t o = static_cast<size_t>(r) * BS + j;
    double v = wy[o] - al * y[o];
    if (y_prev) v -= be * y_prev[o];
    wy[o] = v;
  }
}

// wu = Dinv wy
template <int BS, class TD>
__global__ void judge_dinv_kernel(int nbr, const TD* __restrict__ dinv, const double* __restrict__ wy,
                                  double* __restrict__ wu) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nbr) return;
  const TD* D = dinv + static_cast<size_t>(r) * BS * BS;
  for (int i = 0; i < BS; ++i) {
    double z = 0.0;
    for (int j = 0; j < BS; ++j) z += static_cast<double>(D[i * BS + j]) * wy[static_cast<size_t>(r) * BS + j];
    wu[static_cast<size_t>(r) * BS + i] = z;
  }
}

// partial[c][j] = sum over chunk c of Y_j . w, j < kk (Y_j at Y + j * n)
__global__ __launch_bounds__(256) void multi_dot_kernel(const double* __restrict__ Y, size_t n, int kk,
                                                        const double* __restrict__ w, const int32_t* __restrict__ lo,
                                                        const int32_t* __restrict__ hi, double* __restrict__ partial) {
  __shared__ double lds[2][4];
  const int c = blockIdx.x;
  for (int j = 0; j < kk; ++j) {
    const double* yj = Y + static_cast<size_t>(j) * n;
    double acc = 0.0;
    for (int i = lo[c] + threadIdx.x; i < hi[c]; i += 256) acc = fmadd(yj[i], w[i], acc);
    const double s = block_sum_256(acc, lds[j & 1]);
    if (threadIdx.x == 0) partial[static_cast<size_t>(c) * kk + j] = s;
  }
}

struct OpStoreCoef {
  double* coef;  // [seg][kMaxLanczos]
  __device__ void operator()(int s, int q, double v) const { coef[s * kMaxLanczos + q] = v; }
};

// wu -= sum_j c_j U_j ; wy -= sum_j c_j Y_j (c of the element's segment; off in block rows)
__global__ void judge_reorth_kernel(size_t n, int bs, const int32_t* __restrict__ off, int nseg, int kk,
                                    const double* __restrict__ coef, const double* __restrict__ U,
                                    const double* __restrict__ Y, double* __restrict__ wu, double* __restrict__ wy) {
  const size_t i = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x;
  if (i >= n) return;
  const double* c = coef + seg_of(off, nseg, static_cast<int>(i / bs)) * kMaxLanczos;
  double a = wu[i], b = wy[i];
  for (int j = 0; j < kk; ++j) {
    a -= c[j] * U[static_cast<size_t>(j) * n + i];
    b -= c[j] * Y[static_cast<size_t>(j) * n + i];
  }
  wu[i] = a;
  wy[i] = b;
}

// sc[s].tmp[which] = v
struct OpStoreTmp {
  LevelScalars* sc;
  int which;
  __device__ void operator()(int s, int, double v) const { sc[s].tmp[which] = v; }
};

}  // namespace blk

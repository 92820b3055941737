// Smoothed-aggregation hierarchy, smoother, V-cycle and preconditioned CG
// (paper §2.1, §2.2, §3.1, §4.1), for one problem or a batch of independent ones.
//
// A batch is one block-diagonal operator whose diagonal blocks (instances) are
// coarsened separately: each level keeps its instances as contiguous row ranges,
// the smoothed ones first and the ones whose coarsest level it is last.  One launch
// of each kernel covers every instance of a level; per-instance scalars (Lanczos,
// lambda_hat, Chebyshev coefficients, CG scalars) are indexed by segment; the
// coarsest levels of all instances that end on a level are factored and applied
// together.  Everything in the solve phase stays on the device: the smoother is
// fused into the SpMV kernels, dot products are deterministic two-stage reductions,
// the batched CG keeps its stopping test on the device and can be replayed from a
// captured graph.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "amg_kernels.hpp"
#include "mlp.hpp"
#include "ptap_plan.hpp"
#include "sa_host.hpp"

namespace blk {

// Chunks of a deterministic segmented dot product: chunk c covers scalar rows
// [lo[c], hi[c]) inside one segment; segment s owns chunks [ptr[s], ptr[s+1]).
struct SegGrid {
  int nseg = 0, nchunk = 0;
  DevBuf<int32_t> lo, hi, ptr;
};

struct Level {
  bsr_s* A = nullptr;                  // operator of the level: all its segments
  std::unique_ptr<bsr_s> A_own;        // owned operator (levels >= 1, or F32 copy of A0)
  std::unique_ptr<bsr_s> A_act;        // view of the smoothed prefix (rows [0, act_rows))
  std::unique_ptr<bsr_s> P;            // prolongator: act_rows x (rows of the next level)
  std::vector<int32_t> agg;            // aggregate of each smoothed row (next-level row)
  int32_t n_agg = 0;
  std::vector<int32_t> seg_inst, seg_off;  // instance and block-row range of each segment
  int n_act = 0;                       // segments [0, n_act) smoothed, the rest terminal
  int32_t act_rows = 0;
  int n = 0, bs = 0;                   // scalar dofs, block size
  DevBuf<int32_t> d_act_off;           // block-row offsets of the smoothed segments
  DevBuf<uint16_t> d_row_seg;          // segment of each smoothed row (several segments only)
  SegGrid lgrid;                       // Lanczos dots over the smoothed dofs
  // A P of this level (rows of A_act x rows of the next level), kept by the Galerkin plan
  // of the next level's operator: a view over the plan's arrays (refilled at each use),
  // and the stamps of A and P when the Galerkin pass last formed it (0 = never)
  std::unique_ptr<bsr_s> AP;
  uint64_t ap_stamp = 0, ap_pstamp = 0;
  const int32_t* mir = nullptr;        // symmetric-read mirror index of A (nullptr = full reads)
  int sym_dist = 0;                    // A's typical lower bandwidth (workgroup runs of the symmetric reads)
  DevBuf<char> dinv;                   // [act_rows][bs][bs] hierarchy dtype
  DevBuf<int32_t> diag_idx;
  DevBuf<char> f, out, x, r, d, d2;    // work vectors [rows][vec_nr] (hierarchy dtype)
  int vec_nr = 0;
  DevBuf<double> lz[6];                // Lanczos vectors (F64 hierarchies) ...
  DevBuf<float> lzf[6];                // ... or F32
  // terminal segments: dense inverse Cholesky factors, all concatenated
  int n_term = 0, t_max_rows = 0, t_max_tiles = 0;
  int64_t t_max_nn = 0, t_total = 0;
  DevBuf<int32_t> t_row0, t_nrows, t_ndof, t_dof_off;
  DevBuf<int64_t> t_mat_off;
  DevBuf<double> tL, tY, tYt, tct;
  int n_seg() const { return static_cast<int>(seg_inst.size()); }
};

struct GraphKey {
  const void* x = nullptr;
  const void* A = nullptr;
  int nr = 0, unroll = 0, maxit = 0;
  double rtol = 0.0;
  uint64_t epoch = 0;
  bool operator==(const GraphKey& o) const {
    return x == o.x && A == o.A && nr == o.nr && unroll == o.unroll && maxit == o.maxit && rtol == o.rtol &&
           epoch == o.epoch;
  }
};

}  // namespace blk

struct amg_s {
  blkamg_opts o{};
  int T = BLKAMG_F64;                  // hierarchy dtype
  bsr_s* A0 = nullptr;                 // fine operator (F64, borrowed)
  int n_inst = 1;
  std::vector<int32_t> inst_row0;      // block-row offsets of the instances in A0
  std::vector<std::unique_ptr<blk::Level>> lv;
  blk::DevBuf<blk::LevelScalars> sc;   // [max_levels][n_inst]
  blk::DevBuf<double> partial;         // partial sums of reductions
  blk::DevBuf<double> partial2;
  blk::DevBuf<double> pcg_s;           // single-system CG scalars
  blk::DevBuf<int> flags;              // [0] non-SPD pivot, [1] singular diagonal block
  blk::DevBuf<double> pr, pz, pp, pw;  // CG vectors (F64, [n_dof][nrhs])
  double* host_s = nullptr;            // pinned mirror of the single-system CG scalars
  // batched CG
  blk::SegGrid fgrid[2];               // fine-level dot grids for 1 and 8 right-hand sides
  blk::DevBuf<int32_t> d_fine_dof_off;
  blk::DevBuf<double> bsc;             // [B_FIELDS][n_inst * 8]
  blk::DevBuf<int32_t> bstat;
  int32_t* host_stat = nullptr;
  uint64_t epoch = 1;                  // moves whenever a buffer a captured graph uses moves
  hipStream_t gs = nullptr;            // stream the batched CG graph is captured and run on
  hipEvent_t ev[2] = {nullptr, nullptr};
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  blk::GraphKey gkey;
  // learned eigenbound: model, inference buffers, outcome of the last refresh
  blk::DevBuf<float> model;            // kMlpModel floats
  blk::DevBuf<float> feat, fx, fh1, fh2, fy;
  blk::DevBuf<double> pred_lam, pred_omega;
  std::vector<int> sample_base;        // first sample of each level
  int n_samples = 0;
  std::vector<int32_t> fallback;       // per level: 1 if the last refresh fell back to Lanczos
  std::vector<double> growth;          // [level][inst] A-norm growth of the smoother test
  std::vector<double> omega;           // [level][inst] predicted prolongator weight
  // cold setup: lambda_hat and prolongator weight per [level][inst], and per level
  // whether the network supplied them (1) or Lanczos (0)
  std::vector<double> setup_lam, setup_omega;
  std::vector<int32_t> setup_learned;
  bool user_ops = false;               // operators supplied by the caller (amg_hierarchy_create)
  // BLKAMG_GUARD_PCG: the current smoother scalars come from the network and no test
  // has checked them yet (the next pcg_solve checks its residual, other consumers run
  // the smoother test first); guard_restarts counts the solves restarted by the check
  bool guard_armed = false;
  int32_t guard_restarts = 0;
  void drop_graph() {
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (graph) (void)hipGraphDestroy(graph);
    gexec = nullptr;
    graph = nullptr;
  }
  ~amg_s() {
    if (A0 && !lv.empty() && A0->f32_copy == lv[0]->A) A0->f32_copy = nullptr;
    drop_graph();
    if (gs) (void)hipStreamDestroy(gs);
    for (auto& e : ev)
      if (e) (void)hipEventDestroy(e);
    if (host_s) (void)hipHostFree(host_s);
    if (host_stat) (void)hipHostFree(host_stat);
  }
};

namespace blk {
namespace {

// ---------------------------------------------------------------------------
// Single-system reductions (fused CG path)
// ---------------------------------------------------------------------------
enum RedOp { R_STORE = 0, R_SQRT, R_ALPHA, R_BETA };

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

inline int vgrid(size_t n) { return static_cast<int>((n + 255) / 256); }
inline int rgrid(size_t n) { return static_cast<int>(std::max<size_t>(1, std::min<size_t>((n + 255) / 256, 2048))); }

template <class TV>
TV* buf(DevBuf<char>& b) { return reinterpret_cast<TV*>(b.p); }

size_t tsize(int T) { return T == BLKAMG_F64 ? 8 : 4; }

// ---------------------------------------------------------------------------
// Segmented deterministic dot products
// ---------------------------------------------------------------------------
void build_grid(amg_s* M, SegGrid& g, const std::vector<int64_t>& dof_off, int chunk_rows, int nr) {
  std::vector<int32_t> lo, hi, ptr{0};
  for (size_t t = 0; t + 1 < dof_off.size(); ++t) {
    for (int64_t a = dof_off[t]; a < dof_off[t + 1]; a += chunk_rows) {
      lo.push_back(static_cast<int32_t>(a));
      hi.push_back(static_cast<int32_t>(std::min<int64_t>(a + chunk_rows, dof_off[t + 1])));
    }
    ptr.push_back(static_cast<int32_t>(lo.size()));
  }
  g.nseg = static_cast<int>(dof_off.size()) - 1;
  g.nchunk = static_cast<int>(lo.size());
  upload(g.lo, lo);
  upload(g.hi, hi);
  upload(g.ptr, ptr);
  const size_t need = static_cast<size_t>(g.nchunk) * nr;
  if (M->partial.n < need) {
    HIP_CHECK(hipDeviceSynchronize());
    M->partial.alloc(need);
    M->epoch++;
  }
}

template <int NR, class T, class Op, class TB = T>
void seg_reduce(amg_s* M, const SegGrid& g, const T* a, const TB* b, const Op& op, hipStream_t s) {
  if (g.nseg == 0) return;
  if (g.nchunk > 0) seg_dot_kernel<NR, T, TB><<<g.nchunk, 256, 0, s>>>(a, b, g.lo.p, g.hi.p, M->partial.p);
  seg_finish_kernel<Op><<<g.nseg * NR, 256, 0, s>>>(M->partial.p, g.ptr.p, NR, op);
  HIP_CHECK(hipGetLastError());
}

// ---------------------------------------------------------------------------
// Level layout
// ---------------------------------------------------------------------------
std::unique_ptr<bsr_s> prefix_view(bsr_s* A, int32_t rows) {
  ensure_host_pattern(A);
  auto V = std::make_unique<bsr_s>();
  V->nbr = rows;
  V->nbc = rows;
  V->br = A->br;
  V->bc = A->bc;
  V->dtype = A->dtype;
  V->nnzb = A->h_rowptr[rows];
  V->rowptr = A->rowptr;
  V->colidx = A->colidx;
  V->val = A->val;
  V->h_rowptr.assign(A->h_rowptr.begin(), A->h_rowptr.begin() + rows + 1);
  V->h_colidx.assign(A->h_colidx.begin(), A->h_colidx.begin() + V->nnzb);
  V->h_pattern = true;
  return V;
}

// Derived layout of a level from A, seg_inst, seg_off and n_act: the smoothed view,
// its offsets, the Lanczos grid and the terminal segments' dense-factor layout.
void finalize_level(amg_s* M, Level& L) {
  L.bs = L.A->br;
  L.n = L.A->nbr * L.bs;
  L.act_rows = L.seg_off[L.n_act];
  L.A_act = prefix_view(L.A, L.act_rows);
  std::vector<int32_t> aoff(L.seg_off.begin(), L.seg_off.begin() + L.n_act + 1);
  upload(L.d_act_off, aoff);
  L.d_row_seg.release();
  if (L.n_act > 1) {
    std::vector<uint16_t> rs(static_cast<size_t>(L.act_rows));
    for (int t = 0; t < L.n_act; ++t)
      for (int32_t r = L.seg_off[t]; r < L.seg_off[t + 1]; ++r) rs[r] = static_cast<uint16_t>(t);
    upload(L.d_row_seg, rs);
  }
  std::vector<int64_t> doff;
  for (int t = 0; t <= L.n_act; ++t) doff.push_back(static_cast<int64_t>(L.seg_off[t]) * L.bs);
  build_grid(M, L.lgrid, doff, 8192, kFeatStats);
  const int ns = L.n_seg();
  L.n_term = ns - L.n_act;
  std::vector<int32_t> row0, nrows, ndof, dof_off{0};
  std::vector<int64_t> mat_off{0};
  L.t_max_rows = 0;
  L.t_max_nn = 0;
  for (int t = L.n_act; t < ns; ++t) {
    const int32_t r0 = L.seg_off[t], nr = L.seg_off[t + 1] - L.seg_off[t];
    const int32_t nd = nr * L.bs;
    row0.push_back(r0);
    nrows.push_back(nr);
    ndof.push_back(nd);
    dof_off.push_back(dof_off.back() + nd);
    mat_off.push_back(mat_off.back() + static_cast<int64_t>(nd) * nd);
    L.t_max_rows = std::max(L.t_max_rows, nr);
    L.t_max_nn = std::max<int64_t>(L.t_max_nn, static_cast<int64_t>(nd) * nd);
  }
  mat_off.pop_back();
  L.t_max_tiles = (L.t_max_rows * L.bs + kT - 1) / kT;
  L.t_total = 0;
  for (int t = 0; t < L.n_term; ++t) L.t_total += static_cast<int64_t>(ndof[t]) * ndof[t];
  if (L.n_term > 0) {
    upload(L.t_row0, row0);
    upload(L.t_nrows, nrows);
    upload(L.t_ndof, ndof);
    upload(L.t_dof_off, dof_off);
    upload(L.t_mat_off, mat_off);
    const size_t tot = static_cast<size_t>(std::max<int64_t>(L.t_total, 1));
    L.tL.alloc(tot);
    L.tY.alloc(tot);
    L.tYt.alloc(tot);
  }
}

void ensure_vectors(amg_s* M, int nr) {
  bool grew = false;
  for (auto& lp : M->lv) {
    Level& L = *lp;
    if (L.vec_nr >= nr) continue;
    if (!grew) HIP_CHECK(hipDeviceSynchronize());
    grew = true;
    const size_t ts = tsize(M->T);
    const size_t full = static_cast<size_t>(std::max(L.n, 1)) * nr * ts;
    const size_t act = static_cast<size_t>(std::max(L.act_rows * L.bs, 1)) * nr * ts;
    L.f.alloc(full);
    L.out.alloc(full);
    if (L.n_act > 0) {
      L.x.alloc(act);
      L.r.alloc(act);
      L.d.alloc(act);
      L.d2.alloc(act);
    }
    if (L.n_term > 0) L.tct.alloc(static_cast<size_t>(std::max(L.n, 1)) * nr);
    L.vec_nr = nr;
  }
  if (grew) M->epoch++;
}

// ---------------------------------------------------------------------------
// Smoother data
// ---------------------------------------------------------------------------
void compute_dinv(amg_s* M, Level& L, hipStream_t s) {
  const bsr_s* A = L.A_act.get();
  const int bs = A->br;
  if (A->nbr == 0) return;
  if (!L.dinv.p) {
    L.dinv.alloc(static_cast<size_t>(A->nbr) * bs * bs * tsize(M->T));
    L.diag_idx.alloc(static_cast<size_t>(A->nbr));
  }
  const int grid = vgrid(A->nbr);
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

// k-step Lanczos on D^-1 A in the D inner product, one recurrence per smoothed
// segment of level l; results into sc[l][segment].
template <int BS, class TV>
void lanczos_bs(amg_s* M, int l, hipStream_t s) {
  Level& L = *M->lv[l];
  const bsr_s* A = L.A_act.get();
  const int nbr = A->nbr;
  const size_t n = static_cast<size_t>(nbr) * BS;
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
  int iu_prev = 0, iu = 1, iwu = 2, iy_prev = 3, iy = 4, iwy = 5;  // roles
  LevelScalars* sc = M->sc.p + static_cast<size_t>(l) * M->n_inst;
  const int32_t* off = L.d_act_off.p;
  const int ns = L.n_act;
  const TV* val = static_cast<const TV*>(A->val);
  const TV* dinv = reinterpret_cast<const TV*>(L.dinv.p);
  // start: v -> (u, y) = (v, Dv) / sqrt(v.Dv)
  lanczos_start_kernel<BS, TV, TV><<<vgrid(nbr), 256, 0, s>>>(
      nbr, off, ns, M->o.lanczos_seed + static_cast<uint64_t>(l), val, L.diag_idx.p, V[iwu], V[iwy]);
  HIP_CHECK(hipGetLastError());
  seg_reduce<1>(M, L.lgrid, V[iwu], V[iwy], OpLzSqrt{sc, -1}, s);
  lanczos_scale_kernel<BS, TV><<<vgrid(nbr), 256, 0, s>>>(nbr, off, ns, sc, -1, V[iwu], V[iwy], V[iu], V[iy]);
  HIP_CHECK(hipGetLastError());
  const int k = M->o.lanczos_steps;
  const int G = lanes_for_reads(A, 1, L.mir);
  for (int step = 0; step < k; ++step) {
    EpiLanczos<TV, TV> epi{V[iy_prev], V[iwy], sc, off, ns, step};
    launch_rows<BS, BS, 1, TV, TV, TV>(G, nbr, A->rowptr, A->colidx, val, V[iu], epi, s, L.mir, L.sym_dist);
    seg_reduce<1>(M, L.lgrid, V[iu], V[iwy], OpLzAlpha{sc, step}, s);
    if (step == k - 1) break;
    lanczos_orth_kernel<BS, TV><<<vgrid(nbr), 256, 0, s>>>(nbr, off, ns, sc, step, V[iy], V[iwy], dinv, V[iwu]);
    HIP_CHECK(hipGetLastError());
    seg_reduce<1>(M, L.lgrid, V[iwu], V[iwy], OpLzSqrt{sc, step}, s);
    // (u_prev, u) <- (u, wu/beta) ; (y_prev, y) <- (y, wy/beta)
    lanczos_scale_kernel<BS, TV><<<vgrid(nbr), 256, 0, s>>>(nbr, off, ns, sc, step, V[iwu], V[iwy], V[iu_prev],
                                                            V[iy_prev]);
    HIP_CHECK(hipGetLastError());
    std::swap(iu_prev, iu);
    std::swap(iy_prev, iy);
  }
}

// lambda_hat and Chebyshev coefficients of level l: Lanczos, or the given
// per-segment values (device array, n_act entries) when d_user != NULL.
void refresh_level_scalars(amg_s* M, int l, const double* d_user, hipStream_t s) {
  Level& L = *M->lv[l];
  if (L.n_act == 0) return;
  if (!d_user) {
    const bool f64 = M->T == BLKAMG_F64;
    if (L.bs == 3) { if (f64) lanczos_bs<3, double>(M, l, s); else lanczos_bs<3, float>(M, l, s); }
    else { if (f64) lanczos_bs<6, double>(M, l, s); else lanczos_bs<6, float>(M, l, s); }
  }
  lanczos_finish_kernel<<<(L.n_act + 63) / 64, 64, 0, s>>>(M->sc.p + static_cast<size_t>(l) * M->n_inst, L.n_act,
                                                          M->o.lanczos_steps, d_user, M->o.cheb_lo, M->o.cheb_hi,
                                                          M->o.cheb_degree);
  HIP_CHECK(hipGetLastError());
}

// Dense Cholesky and inverse factor of every terminal segment of L.
void coarse_factor(amg_s* M, Level& L, hipStream_t s) {
  if (L.n_term == 0) return;
  const bsr_s* A = L.A;
  const size_t bytes = static_cast<size_t>(L.t_total) * sizeof(double);
  HIP_CHECK(hipMemsetAsync(L.tL.p, 0, bytes, s));
  HIP_CHECK(hipMemsetAsync(L.tY.p, 0, bytes, s));
  const dim3 eg(std::max(L.t_max_rows, 1), L.n_term);
  if (A->dtype == BLKAMG_F64)
    expand_dense_kernel<double><<<eg, 64, 0, s>>>(L.t_row0.p, L.t_nrows.p, L.t_mat_off.p, L.bs, A->rowptr, A->colidx,
                                                  static_cast<const double*>(A->val), L.tL.p);
  else
    expand_dense_kernel<float><<<eg, 64, 0, s>>>(L.t_row0.p, L.t_nrows.p, L.t_mat_off.p, L.bs, A->rowptr, A->colidx,
                                                 static_cast<const float*>(A->val), L.tL.p);
  HIP_CHECK(hipGetLastError());
  const int nt = L.t_max_tiles;
  for (int k = 0; k < nt; ++k) {
    chol_panel_kernel<<<dim3(nt - k, L.n_term), 256, 0, s>>>(L.tL.p, L.t_mat_off.p, L.t_ndof.p, k, M->flags.p);
    const int m = nt - k - 1;
    if (m > 0) chol_update_kernel<<<dim3(m * (m + 1) / 2, L.n_term), 256, 0, s>>>(L.tL.p, L.t_mat_off.p, L.t_ndof.p, k);
  }
  HIP_CHECK(hipGetLastError());
  tri_inverse_col_kernel<<<dim3(nt, L.n_term), 256, 0, s>>>(L.tL.p, L.tY.p, L.t_mat_off.p, L.t_ndof.p);
  HIP_CHECK(hipGetLastError());
  transpose_dense_kernel<<<dim3(vgrid(static_cast<size_t>(L.t_max_nn)), L.n_term), 256, 0, s>>>(
      L.tY.p, L.tYt.p, L.t_mat_off.p, L.t_ndof.p);
  HIP_CHECK(hipGetLastError());
}

// out = (L L^T)^-1 f = Y^T (Y f) on the terminal rows of the level
template <class TV, int NR>
void coarse_apply(Level& L, const TV* f, TV* out, hipStream_t s) {
  const int rows = L.n - L.act_rows * L.bs;
  if (L.n_term == 0 || rows == 0) return;
  const int g = (rows + 3) / 4;
  const int dof0 = L.act_rows * L.bs;
  dense_tri_batched_kernel<NR, TV, double><<<g, 256, 0, s>>>(L.tY.p, L.t_mat_off.p, L.t_dof_off.p, L.n_term, dof0, 0,
                                                              f, L.tct.p);
  dense_tri_batched_kernel<NR, double, TV><<<g, 256, 0, s>>>(L.tYt.p, L.t_mat_off.p, L.t_dof_off.p, L.n_term, dof0, 1,
                                                              L.tct.p, out);
  HIP_CHECK(hipGetLastError());
}

// The Galerkin pass has just formed the level's A P from its current A and P.
void note_ap(Level& L) {
  L.ap_stamp = L.A->stamp;
  L.ap_pstamp = L.P ? L.P->stamp : 0;
}

// The level's A P when the post-smoothing may update its residual with it: the option
// is on, reading A P costs fewer bytes than reading A (block bytes plus an index each;
// never against the symmetric reads, which read less than either), and A and P still
// hold the values A P was formed from.  nullptr otherwise.  The view is refilled from
// the next level's plan on every call, so it never outlives the arrays it points to.
const bsr_s* ap_for(amg_s* M, int l) {
  Level& L = *M->lv[l];
  if (!M->o.ap_residual || L.bs != 3 || L.mir || !L.P || L.P->bc != 6 || L.n_act == 0 ||
      static_cast<size_t>(l) + 1 >= M->lv.size() || L.A->dtype != M->T)
    return nullptr;
  if (L.ap_stamp != L.A->stamp || L.ap_pstamp != L.P->stamp) return nullptr;
  const auto* pl = static_cast<const PtapPlan*>(M->lv[l + 1]->A->ext.get());
  if (!pl || pl->A != L.A_act.get() || pl->P != L.P.get() || pl->n_ap_rows != L.act_rows || pl->ap_nslots <= 0)
    return nullptr;
  const double vs = static_cast<double>(dtype_size(M->T));
  const double ap_bytes = static_cast<double>(pl->ap_nslots) * (L.bs * L.P->bc * vs + 4.0);
  const double a_bytes = static_cast<double>(L.A_act->nnzb) * (L.bs * L.bs * vs + 4.0);
  if (!(ap_bytes < a_bytes)) return nullptr;
  if (!L.AP) L.AP = std::make_unique<bsr_s>();
  bsr_s* V = L.AP.get();
  V->nbr = pl->n_ap_rows;
  V->nbc = L.P->nbc;
  V->br = L.bs;
  V->bc = L.P->bc;
  V->dtype = M->T;  // A P is formed in the accumulation type, the hierarchy's own
  V->nnzb = pl->ap_nslots;
  V->rowptr = pl->ap_rowptr.p;
  V->colidx = pl->ap_colidx.p;
  V->val = pl->ap_val.p;
  return V;
}

// ---------------------------------------------------------------------------
// V-cycle
// ---------------------------------------------------------------------------
template <int MODE, int NR, class TV>
void smooth(const bsr_s* A, const int32_t* mir, int sym_dist, const TV* gather, const EpiSmooth<MODE, TV, TV>& epi,
            hipStream_t s) {
  const int code = lanes_for_reads(A, NR, mir);
  const auto* v = static_cast<const TV*>(A->val);
  if (A->br == 3) launch_rows<3, 3, NR, TV, TV, TV>(code, A->nbr, A->rowptr, A->colidx, v, gather, epi, s, mir, sym_dist);
  else launch_rows<6, 6, NR, TV, TV, TV>(code, A->nbr, A->rowptr, A->colidx, v, gather, epi, s, mir, sym_dist);
}

template <class TV, int NR>
void vcycle_level(amg_s* M, int l, const TV* f, TV* out, hipStream_t s) {
  Level& L = *M->lv[l];
  coarse_apply<TV, NR>(L, f, out, s);
  if (L.n_act == 0) return;
  const bsr_s* A = L.A_act.get();
  const int nbr = A->nbr;
  const TV* dinv = buf<TV>(L.dinv);
  const LevelScalars* sc = M->sc.p + static_cast<size_t>(l) * M->n_inst;
  const uint16_t* rseg = L.d_row_seg.p;
  TV* x = buf<TV>(L.x);
  TV* r = buf<TV>(L.r);
  TV* d = buf<TV>(L.d);
  TV* d2 = buf<TV>(L.d2);
  const int k = M->o.cheb_degree;
  // pre-smoothing from a zero guess
  TV* first = (k == 1) ? x : d;
  if (L.bs == 3) cheb0_kernel<3, NR, TV><<<vgrid(nbr), 256, 0, s>>>(nbr, rseg, sc, f, dinv, first);
  else cheb0_kernel<6, NR, TV><<<vgrid(nbr), 256, 0, s>>>(nbr, rseg, sc, f, dinv, first);
  HIP_CHECK(hipGetLastError());
  for (int t = 1; t < k; ++t) {
    const bool last = (t == k - 1);
    EpiSmooth<M_STEP, TV, TV> e{t == 1 ? f : r, last ? nullptr : r, d, last ? nullptr : d2, t == 1 ? d : x, x,
                                dinv, sc, rseg, t - 1};
    smooth<M_STEP, NR, TV>(A, L.mir, L.sym_dist, d, e, s);
    std::swap(d, d2);
  }
  // residual and restriction
  {
    EpiSmooth<M_RESID, TV, TV> e{f, r, nullptr, nullptr, nullptr, nullptr, dinv, sc, rseg, 0};
    smooth<M_RESID, NR, TV>(A, L.mir, L.sym_dist, x, e, s);
  }
  Level& C = *M->lv[l + 1];
  TV* fc = buf<TV>(C.f);
  TV* oc = buf<TV>(C.out);
  bsr_s* R = transpose_of(L.P.get(), s);
  spmv(R, 1.0, r, 0.0, fc, M->T, NR, s);
  vcycle_level<TV, NR>(M, l + 1, fc, oc, s);
  spmv(L.P.get(), 1.0, oc, 1.0, x, M->T, NR, s);
  // post-smoothing from x; its first residual f - A x, or, with the Galerkin pass's
  // A P, r - (A P) e_c from the restricted residual still in r (each row's r is read
  // and rewritten by the same lanes; the product gathers only e_c)
  const bsr_s* APv = nullptr;
  if constexpr (NR == 1) APv = ap_for(M, l);
  if (APv) {
    EpiSmooth<M_INITX, TV, TV> e{r, r, nullptr, d, x, out, dinv, sc, rseg, 0};
    launch_rows<3, 6, 1, TV, TV, TV>(lanes_for(APv, 1), APv->nbr, APv->rowptr, APv->colidx,
                                     static_cast<const TV*>(APv->val), oc, e, s);
  } else {
    EpiSmooth<M_INITX, TV, TV> e{f, r, nullptr, d, x, out, dinv, sc, rseg, 0};
    smooth<M_INITX, NR, TV>(A, L.mir, L.sym_dist, x, e, s);
  }
  for (int t = 1; t < k; ++t) {
    const bool last = (t == k - 1);
    EpiSmooth<M_STEP, TV, TV> e{r, last ? nullptr : r, d, last ? nullptr : d2, out, out, dinv, sc, rseg, t - 1};
    smooth<M_STEP, NR, TV>(A, L.mir, L.sym_dist, d, e, s);
    std::swap(d, d2);
  }
}

template <int NR>
void vcycle_nr(amg_s* M, const double* r, double* z, hipStream_t s) {
  Level& L0 = *M->lv[0];
  const size_t n = static_cast<size_t>(L0.n) * NR;
  if (M->T == BLKAMG_F64) {
    vcycle_level<double, NR>(M, 0, r, z, s);
  } else {
    float* f = buf<float>(L0.f);
    float* o = buf<float>(L0.out);
    cast_vec_kernel<double, float><<<vgrid(n), 256, 0, s>>>(n, r, f);
    HIP_CHECK(hipGetLastError());
    vcycle_level<float, NR>(M, 0, f, o, s);
    cast_vec_kernel<float, double><<<vgrid(n), 256, 0, s>>>(n, o, z);
    HIP_CHECK(hipGetLastError());
  }
}

void vcycle(amg_s* M, const double* r, double* z, int nr, hipStream_t s) {
  if (nr == 1) vcycle_nr<1>(M, r, z, s);
  else vcycle_nr<8>(M, r, z, s);
}

// FP32 hierarchy, input already in the fine level's FP32 buffer; returns the FP32
// output buffer (the caller widens it where it reads it)
template <int NR = 1>
const float* vcycle_f32_in_place(amg_s* M, hipStream_t s) {
  Level& L0 = *M->lv[0];
  float* f = buf<float>(L0.f);
  float* o = buf<float>(L0.out);
  vcycle_level<float, NR>(M, 0, f, o, s);
  return o;
}

// ---------------------------------------------------------------------------
// Setup helpers
// ---------------------------------------------------------------------------
// Host strength mask for epsilon > 0 (block Frobenius norms).
std::vector<uint8_t> strength_mask(bsr_s* A, double eps) {
  ensure_host_pattern(A);
  const size_t be = A->block_elems();
  std::vector<double> v = download(static_cast<const double*>(A->val), static_cast<size_t>(A->nnzb) * be);
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
    fail(BLKAMG_ENOTSPD, "a coarsest-level Cholesky met a non-positive pivot");
  }
}

// h_lambda: NULL (Lanczos) or [n_levels - 1][n_inst] user values.
void mlp_refresh(amg_s* M, hipStream_t s);

void smoother_refresh(amg_s* M, const double* h_lambda, hipStream_t s) {
  const int nl = static_cast<int>(M->lv.size());
  if (!h_lambda && M->o.eig_mode == BLKAMG_EIG_MLP && M->model.p) {
    for (int l = 0; l < nl; ++l)
      if (M->lv[l]->n_act > 0) compute_dinv(M, *M->lv[l], s);
    mlp_refresh(M, s);
    for (int l = 0; l < nl; ++l) coarse_factor(M, *M->lv[l], s);
    check_flags(M, s);
    return;
  }
  M->guard_armed = false;
  std::vector<DevBuf<double>> user(static_cast<size_t>(nl));
  for (int l = 0; l < nl; ++l) {
    Level& L = *M->lv[l];
    if (L.n_act > 0) {
      compute_dinv(M, L, s);
      const double* du = nullptr;
      if (h_lambda) {
        std::vector<double> v(static_cast<size_t>(L.n_act));
        for (int t = 0; t < L.n_act; ++t) v[t] = h_lambda[static_cast<size_t>(l) * M->n_inst + L.seg_inst[t]];
        upload(user[l], v);
        du = user[l].p;
      }
      refresh_level_scalars(M, l, du, s);
    }
    coarse_factor(M, L, s);
  }
  check_flags(M, s);  // syncs the stream: the user arrays may be freed after it
}

// ---------------------------------------------------------------------------
// Learned eigenbound: features, reference Lanczos, smoother growth test
// ---------------------------------------------------------------------------
// samples = (level, smoothed segment) pairs, level-major
void map_samples(amg_s* M) {
  const int nl = static_cast<int>(M->lv.size());
  M->sample_base.assign(static_cast<size_t>(nl) + 1, 0);
  for (int l = 0; l < nl; ++l) M->sample_base[l + 1] = M->sample_base[l] + M->lv[l]->n_act;
  M->n_samples = M->sample_base[nl];
}

// features of the smoothed segments of level l into feat[0 .. n_act)[12] (needs Dinv)
void level_features(amg_s* M, int l, float* feat, hipStream_t s) {
  Level& L = *M->lv[l];
  if (L.n_act == 0) return;
  const bsr_s* A = L.A_act.get();
  const SegGrid& g = L.lgrid;
  if (g.nchunk > 0) {
#define BLK_FEAT(BS, T)                                                                                    \
  feature_stats_kernel<BS, T, T><<<g.nchunk, 256, 0, s>>>(A->rowptr, A->colidx, static_cast<const T*>(A->val), \
                                                         reinterpret_cast<const T*>(L.dinv.p), g.lo.p, g.hi.p,  \
                                                         M->partial.p)
    if (M->T == BLKAMG_F64) { if (L.bs == 3) BLK_FEAT(3, double); else BLK_FEAT(6, double); }
    else { if (L.bs == 3) BLK_FEAT(3, float); else BLK_FEAT(6, float); }
#undef BLK_FEAT
    HIP_CHECK(hipGetLastError());
  }
  feature_finish_kernel<<<(L.n_act + 63) / 64, 64, 0, s>>>(M->partial.p, g.ptr.p, L.d_act_off.p, L.n_act, L.bs, l, feat);
  HIP_CHECK(hipGetLastError());
}

void all_features(amg_s* M, float* feat, hipStream_t s) {
  for (size_t l = 0; l < M->lv.size(); ++l)
    level_features(M, static_cast<int>(l), feat + static_cast<size_t>(M->sample_base[l]) * 12, s);
}

template <class TV>
TV* lanczos_vec(Level& L, int t, size_t n) {
  if constexpr (sizeof(TV) == 8) {
    if (L.lz[t].n < n) L.lz[t].alloc(n);
    return reinterpret_cast<TV*>(L.lz[t].p);
  } else {
    if (L.lzf[t].n < n) L.lzf[t].alloc(n);
    return reinterpret_cast<TV*>(L.lzf[t].p);
  }
}

// Largest eigenvalue of the symmetric tridiagonal (alpha[0..m), beta[0..m-1)) by
// Sturm bisection to full precision.
double tridiag_max(const double* alpha, const double* beta, int m) {
  double lo = 1e300, hi = -1e300;
  for (int i = 0; i < m; ++i) {
    const double r = (i > 0 ? std::fabs(beta[i - 1]) : 0.0) + (i < m - 1 ? std::fabs(beta[i]) : 0.0);
    lo = std::min(lo, alpha[i] - r);
    hi = std::max(hi, alpha[i] + r);
  }
  for (int it = 0; it < 300; ++it) {
    const double x = 0.5 * (lo + hi);
    if (x <= lo || x >= hi) break;
    int cnt = 0;
    double q = alpha[0] - x;
    cnt += q < 0;
    for (int i = 1; i < m; ++i) {
      q = alpha[i] - x - beta[i - 1] * beta[i - 1] / (q != 0.0 ? q : 1e-300);
      cnt += q < 0;
    }
    if (cnt == m) hi = x; else lo = x;
  }
  return 0.5 * (lo + hi);
}

// Reference estimate of lambda_max(D^-1 A) per smoothed segment of level l: k steps
// of Lanczos in the D inner product with full reorthogonalisation, FP64 vectors.
template <int BS, class TM>
std::vector<double> judge_level_bs(amg_s* M, int l, int k, hipStream_t s) {
  Level& L = *M->lv[l];
  const bsr_s* A = L.A_act.get();
  const int nbr = A->nbr, ns = L.n_act;
  const size_t n = static_cast<size_t>(nbr) * BS;
  DevBuf<double> U(n * k), Y(n * k), wu(n), wy(n), coef(static_cast<size_t>(ns) * kMaxLanczos);
  DevBuf<LevelScalars> jsc(static_cast<size_t>(ns));
  HIP_CHECK(hipMemsetAsync(jsc.p, 0, jsc.bytes(), s));
  const size_t need = static_cast<size_t>(L.lgrid.nchunk) * k;
  if (M->partial.n < need) {
    HIP_CHECK(hipStreamSynchronize(s));
    M->partial.alloc(need);
    M->epoch++;
  }
  const int32_t* off = L.d_act_off.p;
  const TM* val = static_cast<const TM*>(A->val);
  const TM* dinv = reinterpret_cast<const TM*>(L.dinv.p);
  const int G = lanes_for_reads(A, 1, L.mir);
  lanczos_start_kernel<BS, TM, double><<<vgrid(nbr), 256, 0, s>>>(
      nbr, off, ns, M->o.lanczos_seed + static_cast<uint64_t>(l), val, L.diag_idx.p, wu.p, wy.p);
  seg_reduce<1>(M, L.lgrid, wu.p, wy.p, OpLzSqrt{jsc.p, -1}, s);
  lanczos_scale_kernel<BS, double><<<vgrid(nbr), 256, 0, s>>>(nbr, off, ns, jsc.p, -1, wu.p, wy.p, U.p, Y.p);
  HIP_CHECK(hipGetLastError());
  for (int step = 0; step < k; ++step) {
    double* u = U.p + static_cast<size_t>(step) * n;
    double* y = Y.p + static_cast<size_t>(step) * n;
    launch_rows<BS, BS, 1, TM, double, double>(G, nbr, A->rowptr, A->colidx, val, u,
                                                EpiAxpby<double, double>{wy.p, 1.0, 0.0}, s, L.mir, L.sym_dist);
    seg_reduce<1>(M, L.lgrid, u, wy.p, OpLzAlpha{jsc.p, step}, s);
    if (step == k - 1) break;
    judge_orth_kernel<BS><<<vgrid(nbr), 256, 0, s>>>(nbr, off, ns, jsc.p, step, y, step > 0 ? y - n : nullptr, wy.p);
    judge_dinv_kernel<BS, TM><<<vgrid(nbr), 256, 0, s>>>(nbr, dinv, wy.p, wu.p);
    HIP_CHECK(hipGetLastError());
    const int kk = step + 1;
    if (L.lgrid.nchunk > 0)
      multi_dot_kernel<<<L.lgrid.nchunk, 256, 0, s>>>(Y.p, n, kk, wu.p, L.lgrid.lo.p, L.lgrid.hi.p, M->partial.p);
    seg_finish_kernel<OpStoreCoef><<<ns * kk, 256, 0, s>>>(M->partial.p, L.lgrid.ptr.p, kk, OpStoreCoef{coef.p});
    judge_reorth_kernel<<<vgrid(n), 256, 0, s>>>(n, BS, off, ns, kk, coef.p, U.p, Y.p, wu.p, wy.p);
    HIP_CHECK(hipGetLastError());
    seg_reduce<1>(M, L.lgrid, wu.p, wy.p, OpLzSqrt{jsc.p, step}, s);
    lanczos_scale_kernel<BS, double><<<vgrid(nbr), 256, 0, s>>>(nbr, off, ns, jsc.p, step, wu.p, wy.p, u + n, y + n);
    HIP_CHECK(hipGetLastError());
  }
  std::vector<LevelScalars> h = download(jsc.p, static_cast<size_t>(ns), s);
  std::vector<double> lam(static_cast<size_t>(ns));
  for (int t = 0; t < ns; ++t) {
    int m = std::min(k, (L.seg_off[t + 1] - L.seg_off[t]) * BS);  // no more steps than dofs
    for (int j = 0; j + 1 < m; ++j)
      if (!(h[t].beta[j] > 1e-14 * std::fabs(h[t].alpha[j]))) { m = j + 1; break; }
    lam[t] = tridiag_max(h[t].alpha, h[t].beta, m);
  }
  return lam;
}

std::vector<double> judge_level(amg_s* M, int l, int k, hipStream_t s) {
  Level& L = *M->lv[l];
  if (L.n_act == 0) return {};
  if (M->T == BLKAMG_F64) return L.bs == 3 ? judge_level_bs<3, double>(M, l, k, s) : judge_level_bs<6, double>(M, l, k, s);
  return L.bs == 3 ? judge_level_bs<3, float>(M, l, k, s) : judge_level_bs<6, float>(M, l, k, s);
}

// A-norm growth test of the smoother of level l with its current Chebyshev
// coefficients, as K = growth_steps power steps of the smoother's error propagation S
// (the smoother's result for f = 0): e_0 from splitmix64 (seed kGrowthSeed),
// e_k = S e_(k-1); sc[l][seg].tmp[1] = e_(K-1).A e_(K-1), tmp[2] = e_K.A e_K, so the
// growth is the ratio of the last application, which repeated applications push
// towards the largest |p(lambda)| over the spectrum.
constexpr uint64_t kGrowthSeed = 0xC0FFEE;

template <int BS, class TV>
void growth_level_bs(amg_s* M, int l, hipStream_t s) {
  Level& L = *M->lv[l];
  const bsr_s* A = L.A_act.get();
  const int nbr = A->nbr, ns = L.n_act;
  const size_t n = static_cast<size_t>(nbr) * BS;
  TV* e0 = lanczos_vec<TV>(L, 0, n);
  TV* scratch = lanczos_vec<TV>(L, 1, n);
  TV* w = lanczos_vec<TV>(L, 2, n);
  TV* zero = lanczos_vec<TV>(L, 3, n);
  TV* x = buf<TV>(L.x);
  TV* r = buf<TV>(L.r);
  TV* d = buf<TV>(L.d);
  TV* d2 = buf<TV>(L.d2);
  LevelScalars* sc = M->sc.p + static_cast<size_t>(l) * M->n_inst;
  const int32_t* off = L.d_act_off.p;
  const TV* val = static_cast<const TV*>(A->val);
  const TV* dinv = buf<TV>(L.dinv);
  HIP_CHECK(hipMemsetAsync(zero, 0, n * sizeof(TV), s));
  lanczos_start_kernel<BS, TV, TV><<<vgrid(nbr), 256, 0, s>>>(nbr, off, ns, kGrowthSeed, val, L.diag_idx.p, e0, scratch);
  HIP_CHECK(hipGetLastError());
  const int G = lanes_for_reads(A, 1, L.mir);
  const int K = std::max(1, M->o.growth_steps);
  for (int step = 0; step < K; ++step) {
    if (step > 0) HIP_CHECK(hipMemcpyAsync(e0, x, n * sizeof(TV), hipMemcpyDeviceToDevice, s));
    if (step == K - 1) {
      launch_rows<BS, BS, 1, TV, TV, TV>(G, nbr, A->rowptr, A->colidx, val, e0, EpiAxpby<TV, TV>{w, TV(1), TV(0)}, s,
                                         L.mir, L.sym_dist);
      seg_reduce<1>(M, L.lgrid, e0, w, OpStoreTmp{sc, 1}, s);
    }
    {
      EpiSmooth<M_INITX, TV, TV> e{zero, r, nullptr, d, e0, x, dinv, sc, L.d_row_seg.p, 0};
      smooth<M_INITX, 1, TV>(A, L.mir, L.sym_dist, e0, e, s);
    }
    TV* dd = d;
    TV* dd2 = d2;
    for (int t = 1; t < M->o.cheb_degree; ++t) {
      const bool last = (t == M->o.cheb_degree - 1);
      EpiSmooth<M_STEP, TV, TV> e{r, last ? nullptr : r, dd, last ? nullptr : dd2, x, x, dinv, sc, L.d_row_seg.p,
                                  t - 1};
      smooth<M_STEP, 1, TV>(A, L.mir, L.sym_dist, dd, e, s);
      std::swap(dd, dd2);
    }
  }
  launch_rows<BS, BS, 1, TV, TV, TV>(G, nbr, A->rowptr, A->colidx, val, x, EpiAxpby<TV, TV>{w, TV(1), TV(0)}, s,
                                     L.mir, L.sym_dist);
  seg_reduce<1>(M, L.lgrid, x, w, OpStoreTmp{sc, 2}, s);
}

void growth_level(amg_s* M, int l, hipStream_t s) {
  Level& L = *M->lv[l];
  if (L.n_act == 0) return;
  if (M->T == BLKAMG_F64) { if (L.bs == 3) growth_level_bs<3, double>(M, l, s); else growth_level_bs<6, double>(M, l, s); }
  else { if (L.bs == 3) growth_level_bs<3, float>(M, l, s); else growth_level_bs<6, float>(M, l, s); }
}

// lambda_hat of every smoothed segment from the network: features -> standardise ->
// forward -> lambda, omega; then the Chebyshev coefficients from them, the growth
// test on every level, and Lanczos on every level where some segment's smoother
// grows the A-norm.  Sync.
// Inference buffers for S samples.
void ensure_mlp_buffers(amg_s* M, int S) {
  if (M->feat.n >= static_cast<size_t>(std::max(S, 1)) * 12) return;
  HIP_CHECK(hipDeviceSynchronize());
  const size_t ns = static_cast<size_t>(std::max(S, 1));
  M->feat.alloc(ns * 12);
  M->fx.alloc(ns * 12);
  M->fh1.alloc(ns * kMlpHid);
  M->fh2.alloc(ns * kMlpHid);
  M->fy.alloc(ns * kMlpOut);
  M->pred_lam.alloc(ns);
  M->pred_omega.alloc(ns);
}

// features (already in M->feat[0..S)) -> standardise -> forward -> pred_lam, pred_omega
void mlp_predict(amg_s* M, int S, hipStream_t s) {
  if (S <= 0) return;
  const float* stats = M->model.p + kMlpParams;
  feature_normalize_kernel<<<(S * 12 + 255) / 256, 256, 0, s>>>(S, M->feat.p, stats, M->fx.p);
  HIP_CHECK(hipGetLastError());
  mlp_forward_dev(M->model.p, M->fx.p, S, M->fh1.p, M->fh2.p, M->fy.p, s);
  predict_finish_kernel<<<(S + 255) / 256, 256, 0, s>>>(S, M->fy.p, stats + 24, M->pred_lam.p, M->pred_omega.p);
  HIP_CHECK(hipGetLastError());
}

// A level's smoother from the network fails the guard when some segment's smoother
// grows the A-norm or the predicted lambda_hat is not a positive finite number.
bool growth_fails(const LevelScalars& q, double* g_out) {
  const double g = q.tmp[1] > 0.0 ? std::sqrt(std::max(q.tmp[2], 0.0) / q.tmp[1]) : 0.0;
  if (g_out) *g_out = g;
  return !(g <= 1.0) || !(q.lam > 0.0) || !std::isfinite(q.lam);
}

// The smoother growth test on every smoothed level with the current (network)
// scalars, and Lanczos on each level where some segment fails it.  Sync.
void mlp_check_levels(amg_s* M, hipStream_t s) {
  const int nl = static_cast<int>(M->lv.size());
  for (int l = 0; l < nl; ++l)
    if (M->lv[l]->n_act > 0) growth_level(M, l, s);
  std::vector<LevelScalars> sc = download(M->sc.p, static_cast<size_t>(nl) * M->n_inst, s);
  for (int l = 0; l < nl; ++l) {
    const Level& L = *M->lv[l];
    bool bad = false;
    for (int t = 0; t < L.n_act; ++t) {
      double g = 0.0;
      bad = growth_fails(sc[static_cast<size_t>(l) * M->n_inst + t], &g) || bad;
      M->growth[static_cast<size_t>(l) * M->n_inst + L.seg_inst[t]] = g;
    }
    if (bad) {
      M->fallback[l] = 1;
      refresh_level_scalars(M, l, nullptr, s);
    }
  }
  M->guard_armed = false;
}

// Lanczos on every smoothed level (the residual check of CG failed).
void mlp_fallback_all(amg_s* M, hipStream_t s) {
  const int nl = static_cast<int>(M->lv.size());
  for (int l = 0; l < nl; ++l) {
    if (M->lv[l]->n_act == 0) continue;
    M->fallback[l] = 1;
    refresh_level_scalars(M, l, nullptr, s);
  }
  M->guard_armed = false;
}

void mlp_refresh(amg_s* M, hipStream_t s) {
  BLK_REQUIRE(M->model.p != nullptr, BLKAMG_ESTATE, "eig_mode is MLP but no model was set (amg_set_eig_model)");
  const int nl = static_cast<int>(M->lv.size());
  const int S = M->n_samples;
  ensure_mlp_buffers(M, S);
  all_features(M, M->feat.p, s);
  mlp_predict(M, S, s);
  for (int l = 0; l < nl; ++l) {
    if (M->lv[l]->n_act == 0) continue;
    refresh_level_scalars(M, l, M->pred_lam.p + M->sample_base[l], s);
  }
  std::vector<double> om = download(M->pred_omega.p, static_cast<size_t>(std::max(S, 0)), s);
  M->fallback.assign(static_cast<size_t>(nl), 0);
  M->growth.assign(static_cast<size_t>(nl) * M->n_inst, 0.0);
  M->omega.assign(static_cast<size_t>(nl) * M->n_inst, 0.0);
  for (int l = 0; l < nl; ++l) {
    const Level& L = *M->lv[l];
    for (int t = 0; t < L.n_act; ++t)
      M->omega[static_cast<size_t>(l) * M->n_inst + L.seg_inst[t]] = om[M->sample_base[l] + t];
  }
  // the deferred guard applies to one instance (its CG checks one recurrence)
  if (M->o.mlp_guard == BLKAMG_GUARD_PCG && M->n_inst == 1) M->guard_armed = true;
  else mlp_check_levels(M, s);
}

// Cold setup of level l's smoother scalars and prolongator weights (per smoothed
// segment, into omega_seg): with a model and eig_mode MLP, the network's lambda_hat
// (Chebyshev bounds) and omega (prolongator smoothing), kept when every segment's
// smoother passes the growth test; otherwise, or without a model, Lanczos and
// omega = omega_scale / lambda_hat.  Under the deferred guard (GUARD_PCG, one
// instance) no growth test runs here either: CG checks the smoother scalars, and the
// prolongator weight only shapes the coarse space (any finite positive omega leaves
// the Galerkin operator SPD).  Records both in M->setup_*.  Sync.
void setup_level_scalars(amg_s* M, int l, std::vector<double>& omega_seg, hipStream_t s) {
  Level& L = *M->lv[l];
  const int na = L.n_act;
  omega_seg.assign(static_cast<size_t>(na), 0.0);
  const size_t nrec = static_cast<size_t>(l + 1) * M->n_inst;
  if (M->setup_lam.size() < nrec) {
    M->setup_lam.resize(nrec, 0.0);
    M->setup_omega.resize(nrec, 0.0);
  }
  if (M->setup_learned.size() < static_cast<size_t>(l + 1)) M->setup_learned.resize(static_cast<size_t>(l + 1), 0);
  M->setup_learned[l] = 0;
  if (na == 0) return;
  LevelScalars* scl = M->sc.p + static_cast<size_t>(l) * M->n_inst;
  bool learned = false;
  std::vector<double> om;
  if (M->o.eig_mode == BLKAMG_EIG_MLP && M->model.p) {
    ensure_mlp_buffers(M, na);
    ensure_vectors(M, 1);
    level_features(M, l, M->feat.p, s);
    mlp_predict(M, na, s);
    refresh_level_scalars(M, l, M->pred_lam.p, s);
    const bool deferred = M->o.mlp_guard == BLKAMG_GUARD_PCG && M->n_inst == 1;
    if (!deferred) growth_level(M, l, s);
    std::vector<LevelScalars> q = download(scl, static_cast<size_t>(na), s);
    om = download(M->pred_omega.p, static_cast<size_t>(na), s);
    learned = true;
    for (int t = 0; t < na; ++t)
      learned = learned && (deferred || !growth_fails(q[t], nullptr)) && om[t] > 0.0 && std::isfinite(om[t]) &&
                q[t].lam > 0.0 && std::isfinite(q[t].lam);
  }
  if (!learned) refresh_level_scalars(M, l, nullptr, s);
  std::vector<LevelScalars> q = download(scl, static_cast<size_t>(na), s);
  for (int t = 0; t < na; ++t) {
    omega_seg[t] = learned ? om[t] : M->o.omega_scale / q[t].lam;
    M->setup_lam[static_cast<size_t>(l) * M->n_inst + L.seg_inst[t]] = q[t].lam;
    M->setup_omega[static_cast<size_t>(l) * M->n_inst + L.seg_inst[t]] = omega_seg[t];
  }
  M->setup_learned[l] = learned ? 1 : 0;
}

void galerkin_recompute(amg_s* M, hipStream_t s) {
  if (M->T != BLKAMG_F64) {
    // the FP32 level-0 operator: already written by the COO assembly of the current
    // values, or cast from them here
    bsr_s* A0f = M->lv[0]->A;
    if (!(M->A0->f32_copy == A0f && M->A0->f32_copy_stamp == M->A0->stamp)) {
      cast_values(M->A0->val, BLKAMG_F64, A0f->val, BLKAMG_F32,
                  static_cast<size_t>(M->A0->nnzb) * M->A0->block_elems(), s);
      A0f->stamp++;
    }
  }
  for (size_t l = 0; l + 1 < M->lv.size(); ++l) {
    Level& L = *M->lv[l];
    if (L.n_act == 0) continue;
    const int rc = ptap_numeric(L.A_act.get(), L.P.get(), M->lv[l + 1]->A, s);
    if (rc != BLKAMG_OK) fail(rc, std::string("ptap_numeric: ") + blkamg_last_error());
    note_ap(L);
  }
}

// Copy of a matrix pattern with new (zeroed) values of another dtype.
std::unique_ptr<bsr_s> clone_pattern(bsr_s* A, int dtype) {
  ensure_host_pattern(A);
  return make_owned(A->nbr, A->nbc, A->br, A->bc, dtype, A->h_rowptr, A->h_colidx);
}

// Aggregation of the smoothed segments of L, each instance on its own graph (the
// instances do not couple); local ids are shifted by `base` of the segment.
// Returns per-segment aggregate counts; `agg` gets local ids.
std::vector<int32_t> aggregate_segments(Level& L, const std::vector<uint8_t>& dir, const std::vector<uint8_t>& strong,
                                        std::vector<int32_t>& agg) {
  bsr_s* A = L.A_act.get();
  agg.assign(static_cast<size_t>(L.act_rows), -1);
  std::vector<int32_t> cnt(static_cast<size_t>(L.n_act), 0);
  std::vector<int32_t> rp, ci, la;
  for (int t = 0; t < L.n_act; ++t) {
    const int32_t r0 = L.seg_off[t], r1 = L.seg_off[t + 1];
    const int32_t k0 = A->h_rowptr[r0], k1 = A->h_rowptr[r1];
    const int32_t* prp;
    const int32_t* pci;
    if (r0 == 0 && r1 == A->nbr) {
      prp = A->h_rowptr.data();
      pci = A->h_colidx.data();
    } else {
      rp.resize(static_cast<size_t>(r1 - r0) + 1);
      for (int32_t i = r0; i <= r1; ++i) rp[i - r0] = A->h_rowptr[i] - k0;
      ci.resize(static_cast<size_t>(k1 - k0));
      for (int32_t k = k0; k < k1; ++k) ci[k - k0] = A->h_colidx[k] - r0;
      prp = rp.data();
      pci = ci.data();
    }
    cnt[t] = aggregate_host(r1 - r0, prp, pci, dir.empty() ? nullptr : dir.data() + r0,
                            strong.empty() ? nullptr : strong.data() + k0, la);
    std::copy(la.begin(), la.end(), agg.begin() + r0);
  }
  return cnt;
}

// Aggregation of a one-instance level on the device (Luby rounds); `agg` gets the ids.
std::vector<int32_t> aggregate_level_device(Level& L, const std::vector<uint8_t>& dir, uint64_t seed,
                                            std::vector<int32_t>& agg, hipStream_t s) {
  bsr_s* A = L.A_act.get();
  BLK_REQUIRE(L.n_act == 1 && A->nbr == A->nbc, BLKAMG_EINVAL, "device aggregation takes one instance");
  DevBuf<uint8_t> ddir;
  if (!dir.empty()) upload(ddir, dir);
  DevBuf<int32_t> dagg(static_cast<size_t>(A->nbr));
  int32_t n_agg = 0;
  const int rc = sa_aggregate_device(A, dir.empty() ? nullptr : ddir.p, seed, dagg.p, &n_agg, nullptr, s);
  if (rc != BLKAMG_OK) fail(rc, std::string("sa_aggregate_device: ") + blkamg_last_error());
  agg = download(dagg.p, static_cast<size_t>(A->nbr), s);
  return {n_agg};
}

// Block-diagonal structure check of the instances of A0 (host pattern).
void check_block_diagonal(bsr_s* A, const std::vector<int32_t>& row0) {
  ensure_host_pattern(A);
  for (size_t t = 0; t + 1 < row0.size(); ++t)
    for (int32_t r = row0[t]; r < row0[t + 1]; ++r)
      for (int32_t k = A->h_rowptr[r]; k < A->h_rowptr[r + 1]; ++k) {
        const int32_t c = A->h_colidx[k];
        if (c < row0[t] || c >= row0[t + 1])
          fail(BLKAMG_EINVAL, "A0 couples instance " + std::to_string(t) + " (row " + std::to_string(r) +
                                  ") with column " + std::to_string(c) + " outside it");
      }
}

void autotune_hierarchy(amg_s* M, int nr, hipStream_t s) {
  const int vdt = M->T;
  autotune_lanes(M->A0, BLKAMG_F64, nr, s);
  for (size_t l = 0; l < M->lv.size(); ++l) {
    Level& L = *M->lv[l];
    if (L.n_act == 0) continue;
    autotune_lanes(L.A_act.get(), vdt, nr, s);
    autotune_lanes(L.P.get(), vdt, nr, s);
    autotune_lanes(transpose_of(L.P.get(), s), vdt, nr, s);
  }
}

void check_opts(const blkamg_opts& o) {
  BLK_REQUIRE(o.max_levels >= 1 && o.cheb_degree >= 1 && o.cheb_degree <= kMaxCheb, BLKAMG_EINVAL,
              "bad max_levels or cheb_degree");
  BLK_REQUIRE(o.lanczos_steps >= 2 && o.lanczos_steps <= kMaxLanczos, BLKAMG_EINVAL, "lanczos_steps must be in 2..64");
  BLK_REQUIRE(o.cheb_lo > 0 && o.cheb_hi > o.cheb_lo && o.omega_scale > 0 && o.strength_eps >= 0, BLKAMG_EINVAL,
              "bad smoother parameters");
  BLK_REQUIRE(o.hier_dtype == BLKAMG_F64 || o.hier_dtype == BLKAMG_F32, BLKAMG_EINVAL, "hier_dtype must be F64 or F32");
  BLK_REQUIRE((o.hier_dtype == BLKAMG_F64 && o.p_dtype == BLKAMG_F64) ||
                  (o.hier_dtype == BLKAMG_F32 && (o.p_dtype == BLKAMG_F32 || o.p_dtype == BLKAMG_BF16)),
              BLKAMG_EINVAL, "p_dtype must be F64 for F64 hierarchies and F32/BF16 for F32 hierarchies");
  BLK_REQUIRE(o.pcg_graph_iters >= 0 && o.pcg_graph_iters <= 64, BLKAMG_EINVAL, "pcg_graph_iters must be in 0..64");
  BLK_REQUIRE(o.autotune_nrhs == 0 || o.autotune_nrhs == 1 || o.autotune_nrhs == 8, BLKAMG_EINVAL,
              "autotune_nrhs must be 0, 1 or 8");
  BLK_REQUIRE(o.eig_mode == BLKAMG_EIG_LANCZOS || o.eig_mode == BLKAMG_EIG_MLP, BLKAMG_EINVAL, "bad eig_mode");
  BLK_REQUIRE(o.agg_mode == BLKAMG_AGG_GREEDY || o.agg_mode == BLKAMG_AGG_LUBY, BLKAMG_EINVAL, "bad agg_mode");
  BLK_REQUIRE(o.growth_steps >= 1 && o.growth_steps <= 16, BLKAMG_EINVAL, "growth_steps must be in 1..16");
  BLK_REQUIRE(o.sym_spmv == 0 || o.sym_spmv == 1, BLKAMG_EINVAL, "sym_spmv must be 0 or 1");
  BLK_REQUIRE(o.ap_residual == 0 || o.ap_residual == 1, BLKAMG_EINVAL, "ap_residual must be 0 or 1");
  BLK_REQUIRE(o.mlp_guard == BLKAMG_GUARD_SMOOTHER || o.mlp_guard == BLKAMG_GUARD_PCG, BLKAMG_EINVAL,
              "mlp_guard must be BLKAMG_GUARD_SMOOTHER or BLKAMG_GUARD_PCG");
}

// Validate and copy a model to the device (the caller's array is not kept).
void set_model(amg_s* M, const float* h_model) {
  for (int j = 0; j < 12; ++j)
    BLK_REQUIRE(h_model[kMlpParams + 12 + j] > 0.f, BLKAMG_EINVAL, "feature std must be positive");
  BLK_REQUIRE(h_model[kMlpParams + 26] > 0.f && h_model[kMlpParams + 27] > 0.f, BLKAMG_EINVAL,
              "target std must be positive");
  HIP_CHECK(hipDeviceSynchronize());
  std::vector<float> h(h_model, h_model + kMlpModel);
  upload(M->model, h);
}

// The parts of a hierarchy that do not depend on how its levels were made.
std::unique_ptr<amg_s> new_amg(const blkamg_opts& o, bsr_s* A0, int32_t n_inst, const std::vector<int32_t>& row0) {
  auto M = std::make_unique<amg_s>();
  M->o = o;
  M->T = BLKAMG_F64;  // an F32 hierarchy is derived from the F64 levels at the end of the setup
  M->A0 = A0;
  M->n_inst = n_inst;
  M->inst_row0 = row0;
  M->flags.alloc(4);
  HIP_CHECK(hipMemset(M->flags.p, 0, 4 * sizeof(int)));
  const size_t nsc = static_cast<size_t>(o.max_levels) * n_inst;
  M->sc.alloc(nsc);
  HIP_CHECK(hipMemset(M->sc.p, 0, nsc * sizeof(LevelScalars)));
  M->partial.alloc(static_cast<size_t>(A0->nbr) / 4 + 8192);
  M->partial2.alloc(256);
  M->pcg_s.alloc(S_COUNT);
  HIP_CHECK(hipHostMalloc(reinterpret_cast<void**>(&M->host_s), S_COUNT * sizeof(double)));
  HIP_CHECK(hipHostMalloc(reinterpret_cast<void**>(&M->host_stat), 4 * sizeof(int32_t)));
  M->bstat.alloc(4);
  return M;
}

// Dot grids of the batched CG, solver vectors, learned-part samples, smoother refresh
// and (optionally) the lane autotuner, once the levels exist.
void finish_setup(amg_s* M, hipStream_t s) {
  {
    std::vector<int64_t> doff;
    std::vector<int32_t> d32;
    for (int t = 0; t <= M->n_inst; ++t) {
      doff.push_back(static_cast<int64_t>(M->inst_row0[t]) * M->A0->br);
      d32.push_back(M->inst_row0[t] * M->A0->br);
    }
    build_grid(M, M->fgrid[0], doff, 4096, 1);
    build_grid(M, M->fgrid[1], doff, 512, 8);
    upload(M->d_fine_dof_off, d32);
  }
  ensure_vectors(M, 1);
  map_samples(M);
  // symmetric reads of every smoothed level operator (its prefix view shares the arrays
  // and so the mirror index)
  for (auto& L : M->lv) {
    // FP64 operators only: on FP32 blocks the scattered mirror reads cost more than the
    // bytes they save (fine 3x3 at 128^3: 0.49 ms against 0.45 ms for full reads)
    L->mir = (M->o.sym_spmv && L->n_act > 0 && L->A->dtype == BLKAMG_F64) ? symmetric_mirror(L->A, s) : nullptr;
    L->sym_dist = L->mir ? L->A->sym_dist : 0;
  }
  smoother_refresh(M, nullptr, s);
  if (M->o.autotune_nrhs > 0) autotune_hierarchy(M, M->o.autotune_nrhs, s);
  HIP_CHECK(hipStreamSynchronize(s));
}

amg_s* setup_impl(bsr_t A0, int32_t n_inst, const int32_t* h_row0, const double* h_coords,
                  const uint8_t* h_dirichlet, const blkamg_opts* opts, void* stream) {
  BLK_REQUIRE(A0 != nullptr && h_coords != nullptr, BLKAMG_EINVAL, "NULL argument");
  blkamg_opts o;
  if (opts) o = *opts; else blkamg_opts_default(&o);
  BLK_REQUIRE(A0->dtype == BLKAMG_F64, BLKAMG_EINVAL, "A0 must be F64");
  BLK_REQUIRE(A0->br == 3 && A0->bc == 3 && A0->nbr == A0->nbc, BLKAMG_EINVAL, "A0 must be square with 3x3 blocks");
  BLK_REQUIRE(A0->nbr > 0, BLKAMG_EINVAL, "A0 is empty");
  check_opts(o);
  BLK_REQUIRE(n_inst >= 1 && n_inst <= 65535, BLKAMG_EINVAL, "n_inst must be in 1..65535");
  BLK_REQUIRE(o.agg_mode == BLKAMG_AGG_GREEDY || (n_inst == 1 && o.strength_eps == 0.0), BLKAMG_EINVAL,
              "device aggregation takes one instance and the structural graph (strength_eps = 0)");
  std::vector<int32_t> row0(static_cast<size_t>(n_inst) + 1);
  if (h_row0) {
    std::copy(h_row0, h_row0 + n_inst + 1, row0.begin());
  } else {
    BLK_REQUIRE(n_inst == 1, BLKAMG_EINVAL, "h_inst_row0 is required for n_inst > 1");
    row0 = {0, A0->nbr};
  }
  BLK_REQUIRE(row0[0] == 0 && row0[n_inst] == A0->nbr, BLKAMG_EINVAL, "instance offsets must span A0's rows");
  for (int t = 0; t < n_inst; ++t) BLK_REQUIRE(row0[t + 1] > row0[t], BLKAMG_EINVAL, "empty instance");
  hipStream_t s = as_stream(stream);
  HIP_CHECK(hipStreamSynchronize(s));
  if (n_inst > 1) check_block_diagonal(A0, row0);

  auto M = new_amg(o, A0, n_inst, row0);
  M->o.eig_model = nullptr;  // the caller's array is copied, never kept
  if (o.eig_model) set_model(M.get(), o.eig_model);

  // ---- cold setup in F64 ----
  const int nc_bs = 6;
  auto smoothed = [&](int64_t dofs, int l) { return dofs > o.coarse_eq_limit && l < o.max_levels - 1; };
  {
    auto L0 = std::make_unique<Level>();
    L0->A = A0;
    for (int t = 0; t < n_inst; ++t) {
      L0->seg_inst.push_back(t);
      L0->seg_off.push_back(row0[t]);
    }
    L0->seg_off.push_back(row0[n_inst]);
    int n_act = 0;
    bool seen_term = false;
    for (int t = 0; t < n_inst; ++t) {
      const bool a = smoothed(static_cast<int64_t>(row0[t + 1] - row0[t]) * 3, 0);
      BLK_REQUIRE(!(a && seen_term), BLKAMG_EINVAL,
                  "instances solved directly on the fine level (at most coarse_eq_limit dofs) must come last");
      if (a) ++n_act; else seen_term = true;
    }
    L0->n_act = n_act;
    M->lv.push_back(std::move(L0));
  }
  // near-null space of the current level on the device: the rigid-body modes of the
  // fine nodes, then each level's coarse near-null space
  DevBuf<double> dB(static_cast<size_t>(A0->nbr) * 3 * nc_bs);
  {
    DevBuf<double> dcoords;
    upload(dcoords, std::vector<double>(h_coords, h_coords + static_cast<size_t>(A0->nbr) * 3));
    rigid_body_modes_device(A0->nbr, dcoords.p, dB.p, s);
    HIP_CHECK(hipStreamSynchronize(s));
  }
  std::vector<uint8_t> dir;
  if (h_dirichlet) dir.assign(h_dirichlet, h_dirichlet + A0->nbr);
  for (;;) {
    const int l = static_cast<int>(M->lv.size()) - 1;
    Level& L = *M->lv[l];
    finalize_level(M.get(), L);
    if (L.n_act == 0) break;
    std::vector<uint8_t> strong;
    if (o.strength_eps > 0) strong = strength_mask(L.A_act.get(), o.strength_eps);
    std::vector<int32_t> agg;
    const std::vector<int32_t> cnt = o.agg_mode == BLKAMG_AGG_LUBY
                                         ? aggregate_level_device(L, dir, o.agg_seed, agg, s)
                                         : aggregate_segments(L, dir, strong, agg);
    bool empty = false;
    for (int32_t c : cnt) empty = empty || c == 0;
    if (empty) {
      // nothing to coarsen: with one instance this level becomes the coarsest
      BLK_REQUIRE(n_inst == 1, BLKAMG_EINVAL, "an instance has no aggregates on level " + std::to_string(l));
      L.n_act = 0;
      finalize_level(M.get(), L);
      break;
    }
    // next-level order: instances that are smoothed there first, then the ones it ends
    std::vector<char> next_sm(static_cast<size_t>(L.n_act));
    for (int t = 0; t < L.n_act; ++t) next_sm[t] = smoothed(static_cast<int64_t>(cnt[t]) * nc_bs, l + 1);
    std::vector<int32_t> base(static_cast<size_t>(L.n_act));
    auto next = std::make_unique<Level>();
    int32_t pos = 0;
    for (int pass = 0; pass < 2; ++pass)
      for (int t = 0; t < L.n_act; ++t) {
        if ((next_sm[t] != 0) != (pass == 0)) continue;
        base[t] = pos;
        next->seg_inst.push_back(L.seg_inst[t]);
        next->seg_off.push_back(pos);
        pos += cnt[t];
        if (pass == 0) next->n_act++;
      }
    next->seg_off.push_back(pos);
    const int32_t n_agg = pos;
    for (int t = 0; t < L.n_act; ++t)
      for (int32_t i = L.seg_off[t]; i < L.seg_off[t + 1]; ++i)
        if (agg[i] >= 0) agg[i] += base[t];
    // tentative prolongator: per-aggregate QR on the device (the host QR only for an
    // aggregate too large for the device kernel)
    DevBuf<int32_t> dagg;
    upload(dagg, agg);
    DevBuf<double> dpt(static_cast<size_t>(L.act_rows) * L.bs * nc_bs);
    DevBuf<double> dBc(static_cast<size_t>(n_agg) * nc_bs * nc_bs);
    if (!tentative_device(L.act_rows, L.bs, dagg.p, n_agg, dB.p, dpt.p, dBc.p, s)) {
      std::vector<double> Bh = download(dB.p, static_cast<size_t>(L.act_rows) * L.bs * nc_bs, s);
      std::vector<double> Pt, Bc;
      tentative_host(L.act_rows, L.bs, nc_bs, agg, n_agg, Bh, Pt, Bc);
      upload(dpt, Pt);
      upload(dBc, Bc);
    }
    L.agg = std::move(agg);
    L.n_agg = n_agg;
    compute_dinv(M.get(), L, s);
    check_flags(M.get(), s);
    std::vector<double> omega_seg;
    setup_level_scalars(M.get(), l, omega_seg, s);
    // smoothed prolongator: pattern of A P~ (structural product on the device, or on the
    // host for rows beyond the device product's limit), values on the device
    bsr_s* A = L.A_act.get();
    std::vector<int32_t> ptrp(static_cast<size_t>(A->nbr) + 1, 0), ptci;
    for (int32_t i = 0; i < A->nbr; ++i) {
      if (L.agg[i] >= 0) ptci.push_back(L.agg[i]);
      ptrp[i + 1] = static_cast<int32_t>(ptci.size());
    }
    {
      DevBuf<int32_t> dtrp, dtci, prp_d, pci_d;
      upload(dtrp, ptrp);
      upload(dtci, ptci);
      int64_t pnnz = 0;
      if (structural_product_device(A->nbr, n_agg, A->rowptr, A->colidx, dtrp.p, dtci.p, prp_d, pci_d, pnnz, s)) {
        L.P = make_owned_device(A->nbr, n_agg, A->br, nc_bs, BLKAMG_F64, std::move(prp_d), std::move(pci_d), pnnz, s);
      } else {
        std::vector<int32_t> prp, pci;
        structural_product_host(A->nbr, A->h_rowptr, A->h_colidx, n_agg, ptrp, ptci, prp, pci);
        L.P = make_owned(A->nbr, n_agg, A->br, nc_bs, BLKAMG_F64, std::move(prp), std::move(pci));
      }
    }
    {
      DevBuf<double> dom;
      upload(dom, omega_seg);
      const int64_t nnz = L.P->nnzb;
      if (nnz > 0) {
        const int grid = static_cast<int>((nnz + 255) / 256);
#define BLK_SMOOTHP(BS)                                                                                          \
  smooth_p_kernel<BS, 6><<<grid, 256, 0, s>>>(A->nbr, A->rowptr, A->colidx, static_cast<const double*>(A->val),  \
                                              dagg.p, dpt.p, reinterpret_cast<const double*>(L.dinv.p),          \
                                              L.d_act_off.p, L.n_act, dom.p, L.P->rowptr,                       \
                                              L.P->colidx, static_cast<double*>(L.P->val))
        if (A->br == 3) BLK_SMOOTHP(3); else BLK_SMOOTHP(6);
#undef BLK_SMOOTHP
        HIP_CHECK(hipGetLastError());
      }
      HIP_CHECK(hipStreamSynchronize(s));  // dom (and dagg / dpt below) are freed at scope exit
    }
    bsr_t Cm = nullptr;
    int rc = ptap_symbolic_ex(A, L.P.get(), BLKAMG_PTAP_SYMMETRIC, &Cm, stream);
    if (rc != BLKAMG_OK) fail(rc, std::string("ptap_symbolic: ") + blkamg_last_error());
    next->A_own.reset(Cm);
    next->A = Cm;
    rc = ptap_numeric(A, L.P.get(), Cm, stream);
    if (rc != BLKAMG_OK) fail(rc, std::string("ptap_numeric: ") + blkamg_last_error());
    note_ap(L);
    dB = std::move(dBc);
    dir.clear();
    M->lv.push_back(std::move(next));
  }
  const int nl = static_cast<int>(M->lv.size());

  // ---- derive the F32 hierarchy: A_l and P_l stored in F32 (P optionally BF16) ----
  if (o.hier_dtype == BLKAMG_F32) {
    std::unique_ptr<bsr_s> Af = clone_pattern(A0, BLKAMG_F32);
    cast_values(A0->val, BLKAMG_F64, Af->val, BLKAMG_F32, static_cast<size_t>(A0->nnzb) * 9, s);
    for (int l = 0; l < nl; ++l) {
      Level& L = *M->lv[l];
      L.A_own = std::move(Af);  // frees this level's F64 operator
      L.A = L.A_own.get();
      L.A_act = prefix_view(L.A, L.act_rows);
      L.dinv.release();
      L.diag_idx.release();
      for (auto& v : L.lz) v.release();
      if (l + 1 < nl && L.n_act > 0) {
        bsr_s* P64 = L.P.get();
        std::unique_ptr<bsr_s> Pf = clone_pattern(P64, o.p_dtype);
        cast_values(P64->val, BLKAMG_F64, Pf->val, o.p_dtype, static_cast<size_t>(P64->nnzb) * P64->block_elems(), s);
        bsr_t Cm = nullptr;
        int rc = ptap_symbolic_ex(L.A_act.get(), Pf.get(), BLKAMG_PTAP_SYMMETRIC, &Cm, stream);
        if (rc != BLKAMG_OK) fail(rc, std::string("ptap_symbolic: ") + blkamg_last_error());
        Af.reset(Cm);
        rc = ptap_numeric(L.A_act.get(), Pf.get(), Cm, stream);
        if (rc != BLKAMG_OK) fail(rc, std::string("ptap_numeric: ") + blkamg_last_error());
        HIP_CHECK(hipStreamSynchronize(s));
        L.P = std::move(Pf);
        note_ap(L);
      }
    }
    M->T = BLKAMG_F32;
    // the assembly of A0 writes this level-0 copy beside the values from now on (the
    // latest such hierarchy on A0; the others cast at their recompute)
    A0->f32_copy = M->lv[0]->A;
    A0->f32_copy_stamp = A0->stamp;
  }
  finish_setup(M.get(), s);
  return M.release();
}

Level* get_level(amg_s* M, int32_t l) {
  BLK_REQUIRE(M != nullptr, BLKAMG_EINVAL, "M is NULL");
  BLK_REQUIRE(l >= 0 && l < static_cast<int32_t>(M->lv.size()), BLKAMG_EINVAL, "level out of range");
  return M->lv[l].get();
}

// ---------------------------------------------------------------------------
// CG
// ---------------------------------------------------------------------------
// One system, one right-hand side: the SpMV with the p.w dot fused in, one 8-byte
// read per iteration for the stopping test.
int pcg_single(bsr_s* A, amg_s* M, const double* d_b, double* d_x, double rtol, int32_t maxit, int32_t* iters,
               double* relres, hipStream_t s) {
  const size_t n = static_cast<size_t>(M->lv[0]->n);
  if (M->pr.n < n) {
    HIP_CHECK(hipStreamSynchronize(s));
    M->pr.alloc(n);
    M->pz.alloc(n);
    M->pp.alloc(n);
    M->pw.alloc(n);
    M->epoch++;
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
  // With an FP32 hierarchy the residual update also writes the V-cycle's FP32 input and
  // the dot and direction updates read its FP32 output: no separate casts.
  const bool mixed = M->T == BLKAMG_F32;
  float* r32 = mixed ? buf<float>(M->lv[0]->f) : nullptr;
  auto precondition = [&]() {
    if (mixed) {
      const float* z32 = vcycle_f32_in_place(M, s);
      dot_kernel<float><<<vg, 256, 0, s>>>(n, r, z32, M->partial.p);
      return z32;
    }
    vcycle(M, r, z, 1, s);
    dot_kernel<double><<<vg, 256, 0, s>>>(n, r, z, M->partial.p);
    return static_cast<const float*>(nullptr);
  };
  auto direction = [&](const float* z32, int use_beta) {
    if (mixed) pcg_p_kernel<float><<<vgrid(n), 256, 0, s>>>(n, sc, use_beta, z32, p);
    else pcg_p_kernel<double><<<vgrid(n), 256, 0, s>>>(n, sc, use_beta, z, p);
    HIP_CHECK(hipGetLastError());
  };
  if (mixed) {
    cast_vec_kernel<double, float><<<vgrid(n), 256, 0, s>>>(n, r, r32);
    HIP_CHECK(hipGetLastError());
  }
  {
    const float* z32 = precondition();
    HIP_CHECK(hipGetLastError());
    reduce(M, vg, sc + S_RZ, R_STORE, s);
    direction(z32, 0);
  }
  const int32_t* mir = M->o.sym_spmv ? symmetric_mirror(A, s) : nullptr;
  const int G = lanes_for_reads(A, 1, mir);
  bool converged = false;
  // deferred guard of network scalars: the preconditioned r.z must stay positive and the
  // residual must not grow far above its smallest value (a smoother whose Chebyshev
  // interval misses the top of the spectrum makes the V-cycle indefinite)
  const bool guard = M->guard_armed;
  constexpr double kGuardGrowth = 1e3;
  double rmin = bn;
  while (it < maxit) {
    EpiPcgW epi{p, w, M->partial.p};
    const int sg = A->br == 3 ? launch_rows<3, 3, 1, double, double, double>(G, A->nbr, A->rowptr, A->colidx,
                                                                            static_cast<const double*>(A->val), p, epi, s,
                                                                            mir, A->sym_dist)
                              : launch_rows<6, 6, 1, double, double, double>(G, A->nbr, A->rowptr, A->colidx,
                                                                            static_cast<const double*>(A->val), p, epi, s,
                                                                            mir, A->sym_dist);
    reduce(M, sg, nullptr, R_ALPHA, s);
    pcg_update_kernel<<<vg, 256, 0, s>>>(n, sc, p, w, d_x, r, M->partial.p, r32);
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
    if (guard && (!(M->host_s[S_RZ] > 0.0) || !std::isfinite(rn) || rn > kGuardGrowth * rmin)) {
      mlp_fallback_all(M, s);
      M->guard_restarts++;
      return pcg_single(A, M, d_b, d_x, rtol, maxit, iters, relres, s);
    }
    rmin = std::min(rmin, rn);
    if (rn <= rtol * bn) { converged = true; break; }
    const float* z32 = precondition();
    HIP_CHECK(hipGetLastError());
    reduce(M, vg, nullptr, R_BETA, s);
    direction(z32, 1);
  }
  if (iters) *iters = it;
  if (relres) *relres = rn / bn;
  return converged ? BLKAMG_OK : BLKAMG_ENOCONV;
}

// Batched CG: one recurrence per (instance, right-hand side) with its own stopping
// test kept on the device; a stopped system is frozen (alpha = 0).
template <int NR>
void bpcg_iteration(amg_s* M, bsr_s* A, double* x, double rtol, int maxit, hipStream_t s) {
  const size_t nrow = static_cast<size_t>(M->lv[0]->n);
  const int nseg = M->n_inst;
  const int stride = nseg * NR;
  double* bs = M->bsc.p;
  const SegGrid& g = M->fgrid[NR == 1 ? 0 : 1];
  const int32_t* off = M->d_fine_dof_off.p;
  double* r = M->pr.p;
  double* z = M->pz.p;
  double* p = M->pp.p;
  double* w = M->pw.p;
  const int vg = vgrid(nrow * NR);
  spmv(A, 1.0, p, 0.0, w, BLKAMG_F64, NR, s);
  seg_reduce<NR>(M, g, p, w, OpBAlpha{bs, stride, NR}, s);
  // with an FP32 hierarchy the update writes the V-cycle's FP32 input and the reads of
  // its output widen FP32 values (no separate casts)
  const bool mixed = M->T == BLKAMG_F32;
  float* r32 = mixed ? buf<float>(M->lv[0]->f) : nullptr;
  bpcg_axpy_kernel<<<vg, 256, 0, s>>>(nrow, NR, off, nseg, bs, stride, p, w, x, r, r32);
  HIP_CHECK(hipGetLastError());
  seg_reduce<NR>(M, g, r, r, OpBRr{bs, stride, NR, maxit, rtol}, s);
  if (mixed) {
    const float* z32 = vcycle_f32_in_place<NR>(M, s);
    seg_reduce<NR>(M, g, r, z32, OpBBeta{bs, stride, NR}, s);
    bpcg_p_kernel<float><<<vg, 256, 0, s>>>(nrow, NR, off, nseg, bs, stride, 1, z32, p);
  } else {
    vcycle(M, r, z, NR, s);
    seg_reduce<NR>(M, g, r, z, OpBBeta{bs, stride, NR}, s);
    bpcg_p_kernel<double><<<vg, 256, 0, s>>>(nrow, NR, off, nseg, bs, stride, 1, z, p);
  }
  HIP_CHECK(hipGetLastError());
}

template <int NR>
void bpcg_block(amg_s* M, bsr_s* A, double* x, double rtol, int maxit, int U, hipStream_t s) {
  for (int u = 0; u < U; ++u) bpcg_iteration<NR>(M, A, x, rtol, maxit, s);
  bpcg_status_kernel<<<1, 64, 0, s>>>(M->bsc.p, M->n_inst * NR, M->n_inst * NR, M->bstat.p);
  HIP_CHECK(hipGetLastError());
}

// Capture U iterations plus the status kernel as a graph on M->gs (reused while the
// key matches).  The capture enqueues no memset and no allocation.
template <int NR>
void bpcg_graph(amg_s* M, bsr_s* A, double* x, double rtol, int maxit, int U) {
  GraphKey key;
  key.x = x;
  key.A = A;
  key.nr = NR;
  key.unroll = U;
  key.maxit = maxit;
  key.rtol = rtol;
  key.epoch = M->epoch;
  if (M->gexec && key == M->gkey) return;
  M->drop_graph();
  HIP_CHECK(hipStreamBeginCapture(M->gs, hipStreamCaptureModeThreadLocal));
  try {
    bpcg_block<NR>(M, A, x, rtol, maxit, U, M->gs);
  } catch (...) {
    hipGraph_t g = nullptr;
    (void)hipStreamEndCapture(M->gs, &g);
    if (g) (void)hipGraphDestroy(g);
    throw;
  }
  HIP_CHECK(hipStreamEndCapture(M->gs, &M->graph));
  HIP_CHECK(hipGraphInstantiate(&M->gexec, M->graph, nullptr, nullptr, 0));
  M->gkey = key;
}

template <int NR>
int pcg_batched(bsr_s* A, amg_s* M, const double* d_b, double* d_x, double rtol, int32_t maxit, int32_t* iters,
                double* relres, hipStream_t s) {
  const size_t nrow = static_cast<size_t>(M->lv[0]->n);
  const size_t n = nrow * NR;
  const int nsys = M->n_inst * NR;
  ensure_vectors(M, NR);
  if (M->pr.n < n) {
    HIP_CHECK(hipDeviceSynchronize());
    M->pr.alloc(n);
    M->pz.alloc(n);
    M->pp.alloc(n);
    M->pw.alloc(n);
    M->epoch++;
  }
  if (M->bsc.n < static_cast<size_t>(B_FIELDS) * nsys) {
    HIP_CHECK(hipDeviceSynchronize());
    M->bsc.alloc(static_cast<size_t>(B_FIELDS) * M->n_inst * 8);
    M->epoch++;
  }
  const int U = M->o.pcg_graph_iters;
  const bool use_graph = U > 0;
  if (use_graph && !M->gs) {
    HIP_CHECK(hipStreamCreateWithFlags(&M->gs, hipStreamNonBlocking));
    HIP_CHECK(hipEventCreateWithFlags(&M->ev[0], hipEventDisableTiming));
    HIP_CHECK(hipEventCreateWithFlags(&M->ev[1], hipEventDisableTiming));
  }
  const int stride = nsys;
  double* bs = M->bsc.p;
  const SegGrid& g = M->fgrid[NR == 1 ? 0 : 1];
  const int32_t* off = M->d_fine_dof_off.p;
  // start: r = b, x = 0, z = M r, p = z
  bpcg_init_kernel<<<vgrid(n), 256, 0, s>>>(n, d_b, d_x, M->pr.p);
  HIP_CHECK(hipGetLastError());
  seg_reduce<NR>(M, g, d_b, d_b, OpBInit{bs, stride, NR, maxit}, s);
  if (M->T == BLKAMG_F32) {
    cast_vec_kernel<double, float><<<vgrid(n), 256, 0, s>>>(n, M->pr.p, buf<float>(M->lv[0]->f));
    HIP_CHECK(hipGetLastError());
    const float* z32 = vcycle_f32_in_place<NR>(M, s);
    seg_reduce<NR>(M, g, M->pr.p, z32, OpBRz0{bs, stride, NR}, s);
    bpcg_p_kernel<float><<<vgrid(n), 256, 0, s>>>(nrow, NR, off, M->n_inst, bs, stride, 0, z32, M->pp.p);
  } else {
    vcycle(M, M->pr.p, M->pz.p, NR, s);
    seg_reduce<NR>(M, g, M->pr.p, M->pz.p, OpBRz0{bs, stride, NR}, s);
    bpcg_p_kernel<double><<<vgrid(n), 256, 0, s>>>(nrow, NR, off, M->n_inst, bs, stride, 0, M->pz.p, M->pp.p);
  }
  HIP_CHECK(hipGetLastError());
  bpcg_status_kernel<<<1, 64, 0, s>>>(bs, stride, nsys, M->bstat.p);
  HIP_CHECK(hipGetLastError());
  hipStream_t ls = s;
  if (use_graph) {
    bpcg_graph<NR>(M, A, d_x, rtol, maxit, U);
    HIP_CHECK(hipEventRecord(M->ev[0], s));
    HIP_CHECK(hipStreamWaitEvent(M->gs, M->ev[0], 0));
    ls = M->gs;
  }
  HIP_CHECK(hipMemcpyAsync(M->host_stat, M->bstat.p, 2 * sizeof(int32_t), hipMemcpyDeviceToHost, ls));
  HIP_CHECK(hipStreamSynchronize(ls));
  const int step = use_graph ? U : 1;
  for (int64_t done_its = 0; M->host_stat[0] > 0 && done_its < static_cast<int64_t>(maxit) + step; done_its += step) {
    if (use_graph) HIP_CHECK(hipGraphLaunch(M->gexec, M->gs));
    else bpcg_block<NR>(M, A, d_x, rtol, maxit, 1, s);
    HIP_CHECK(hipMemcpyAsync(M->host_stat, M->bstat.p, 2 * sizeof(int32_t), hipMemcpyDeviceToHost, ls));
    HIP_CHECK(hipStreamSynchronize(ls));
  }
  if (use_graph) {
    HIP_CHECK(hipEventRecord(M->ev[1], M->gs));
    HIP_CHECK(hipStreamWaitEvent(s, M->ev[1], 0));
  }
  std::vector<double> h = download(bs, static_cast<size_t>(B_FIELDS) * stride, s);
  bool any_brk = false, any_noconv = false;
  for (int k = 0; k < nsys; ++k) {
    const double bb = h[B_BB * stride + k], rr = h[B_RR * stride + k], dn = h[B_DONE * stride + k];
    if (iters) iters[k] = static_cast<int32_t>(h[B_ITS * stride + k]);
    if (relres) relres[k] = bb > 0.0 ? std::sqrt(rr / bb) : 0.0;
    any_brk = any_brk || dn == 2.0;
    any_noconv = any_noconv || dn == 3.0 || dn == 0.0;
  }
  if (any_brk) fail(BLKAMG_EBREAKDOWN, "CG breakdown: p^T A p <= 0 in at least one system");
  return any_noconv ? BLKAMG_ENOCONV : BLKAMG_OK;
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
  o->pcg_graph_iters = 4;
  o->autotune_nrhs = 0;
  o->eig_mode = BLKAMG_EIG_LANCZOS;
  o->agg_mode = BLKAMG_AGG_GREEDY;
  o->agg_seed = 0x4D495332ull;
  o->growth_steps = 3;
  o->eig_model = nullptr;
  o->mlp_guard = BLKAMG_GUARD_SMOOTHER;
  o->sym_spmv = 1;
  o->ap_residual = 1;
}

int amg_setup(bsr_t A0, const double* h_coords, const uint8_t* h_dirichlet, const blkamg_opts* opts, void* stream,
              amg_t* out) {
  BLK_API_BEGIN
  BLK_REQUIRE(out != nullptr, BLKAMG_EINVAL, "NULL argument");
  *out = nullptr;
  *out = setup_impl(A0, 1, nullptr, h_coords, h_dirichlet, opts, stream);
  BLK_API_END
}

int amg_setup_batched(bsr_t A0, int32_t n_inst, const int32_t* h_inst_row0, const double* h_coords,
                      const uint8_t* h_dirichlet, const blkamg_opts* opts, void* stream, amg_t* out) {
  BLK_API_BEGIN
  BLK_REQUIRE(out != nullptr && h_inst_row0 != nullptr, BLKAMG_EINVAL, "NULL argument");
  *out = nullptr;
  *out = setup_impl(A0, n_inst, h_inst_row0, h_coords, h_dirichlet, opts, stream);
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

int amg_num_instances(amg_t M, int32_t* n_inst) {
  BLK_API_BEGIN
  BLK_REQUIRE(M != nullptr && n_inst != nullptr, BLKAMG_EINVAL, "NULL argument");
  *n_inst = M->n_inst;
  BLK_API_END
}

int amg_level(amg_t M, int32_t level, bsr_t* A, bsr_t* P) {
  BLK_API_BEGIN
  Level* L = get_level(M, level);
  if (A) *A = L->A;
  if (P) *P = L->P.get();
  BLK_API_END
}

int amg_instance_rows(amg_t M, int32_t level, int32_t* h_row0, int32_t* h_nrows, int32_t* h_state) {
  BLK_API_BEGIN
  Level* L = get_level(M, level);
  for (int t = 0; t < M->n_inst; ++t) {
    if (h_row0) h_row0[t] = 0;
    if (h_nrows) h_nrows[t] = 0;
    if (h_state) h_state[t] = 0;
  }
  for (int t = 0; t < L->n_seg(); ++t) {
    const int i = L->seg_inst[t];
    if (h_row0) h_row0[i] = L->seg_off[t];
    if (h_nrows) h_nrows[i] = L->seg_off[t + 1] - L->seg_off[t];
    if (h_state) h_state[i] = t < L->n_act ? 1 : 2;
  }
  BLK_API_END
}

int amg_aggregates(amg_t M, int32_t level, int32_t* h_agg) {
  BLK_API_BEGIN
  Level* L = get_level(M, level);
  BLK_REQUIRE(L->n_act > 0, BLKAMG_EINVAL, "the level has no smoothed rows");
  BLK_REQUIRE(!M->user_ops, BLKAMG_EINVAL, "no aggregates: the prolongators were supplied by the caller");
  BLK_REQUIRE(h_agg != nullptr, BLKAMG_EINVAL, "h_agg is NULL");
  std::copy(L->agg.begin(), L->agg.end(), h_agg);
  BLK_API_END
}

int amg_lambdas(amg_t M, double* h_lam) {
  BLK_API_BEGIN
  BLK_REQUIRE(M != nullptr && h_lam != nullptr, BLKAMG_EINVAL, "NULL argument");
  const size_t nl = M->lv.size();
  std::vector<LevelScalars> sc = download(M->sc.p, nl * M->n_inst);
  for (size_t l = 0; l + 1 < nl; ++l) {
    for (int t = 0; t < M->n_inst; ++t) h_lam[l * M->n_inst + t] = 0.0;
    const Level& L = *M->lv[l];
    for (int t = 0; t < L.n_act; ++t) h_lam[l * M->n_inst + L.seg_inst[t]] = sc[l * M->n_inst + t].lam;
  }
  BLK_API_END
}

int amg_galerkin_recompute(amg_t M, void* stream) {
  BLK_API_BEGIN
  BLK_REQUIRE(M != nullptr, BLKAMG_EINVAL, "M is NULL");
  BLK_REQUIRE(!M->user_ops, BLKAMG_EINVAL,
              "the coarse operators belong to the caller: recompute them with ptap_numeric, then amg_hierarchy_update");
  galerkin_recompute(M, as_stream(stream));
  BLK_API_END
}

int amg_hierarchy_create(int32_t n_levels, const bsr_t* A, const bsr_t* P, const blkamg_opts* opts, void* stream,
                         amg_t* out) {
  BLK_API_BEGIN
  BLK_REQUIRE(out != nullptr && A != nullptr, BLKAMG_EINVAL, "NULL argument");
  *out = nullptr;
  blkamg_opts o;
  if (opts) o = *opts; else blkamg_opts_default(&o);
  check_opts(o);
  BLK_REQUIRE(o.hier_dtype == BLKAMG_F64, BLKAMG_EINVAL, "caller-supplied operators are used in F64: hier_dtype must be F64");
  BLK_REQUIRE(n_levels >= 1 && n_levels <= o.max_levels, BLKAMG_EINVAL, "n_levels must be in 1..max_levels");
  BLK_REQUIRE(n_levels == 1 || P != nullptr, BLKAMG_EINVAL, "P is NULL");
  for (int l = 0; l < n_levels; ++l) {
    const bsr_s* a = A[l];
    BLK_REQUIRE(a != nullptr && a->dtype == BLKAMG_F64 && a->br == a->bc && a->nbr == a->nbc && a->nbr > 0,
                BLKAMG_EINVAL, "A[" + std::to_string(l) + "] must be a non-empty square-blocked F64 operator");
    BLK_REQUIRE(l == 0 ? a->br == 3 : a->br == 6, BLKAMG_EINVAL,
                "A[0] must have 3x3 blocks and coarser levels 6x6 blocks");
    if (l + 1 < n_levels) {
      const bsr_s* p = P[l];
      BLK_REQUIRE(p != nullptr && p->dtype == BLKAMG_F64 && p->nbr == a->nbr && p->br == a->br && p->bc == 6 &&
                      p->nbc == A[l + 1]->nbr,
                  BLKAMG_EINVAL, "P[" + std::to_string(l) + "] must be F64, A[l].nbr x A[l+1].nbr, blocks bs x 6");
    }
  }
  hipStream_t s = as_stream(stream);
  HIP_CHECK(hipStreamSynchronize(s));
  const std::vector<int32_t> row0{0, A[0]->nbr};
  auto M = new_amg(o, A[0], 1, row0);
  M->user_ops = true;
  M->o.eig_model = nullptr;  // the caller's array is copied, never kept
  if (o.eig_model) set_model(M.get(), o.eig_model);
  for (int l = 0; l < n_levels; ++l) {
    auto L = std::make_unique<Level>();
    L->A = A[l];
    L->seg_inst = {0};
    L->seg_off = {0, A[l]->nbr};
    L->n_act = l + 1 < n_levels ? 1 : 0;
    finalize_level(M.get(), *L);
    if (l + 1 < n_levels) {
      // the library keeps its own copy of the prolongator values and pattern
      bsr_s* p = P[l];
      ensure_host_pattern(p);
      std::vector<int32_t> rp = p->h_rowptr, ci = p->h_colidx;
      L->P = make_owned(p->nbr, p->nbc, p->br, p->bc, BLKAMG_F64, std::move(rp), std::move(ci));
      HIP_CHECK(hipMemcpyAsync(L->P->val, p->val, p->val_bytes(), hipMemcpyDeviceToDevice, s));
      L->n_agg = A[l + 1]->nbr;
    }
    M->lv.push_back(std::move(L));
  }
  finish_setup(M.get(), s);
  *out = M.release();
  BLK_API_END
}

int amg_hierarchy_update(amg_t M, const float* h_lambda, void* stream) {
  BLK_API_BEGIN
  BLK_REQUIRE(M != nullptr, BLKAMG_EINVAL, "M is NULL");
  std::vector<double> lam;
  if (h_lambda) {
    lam.assign(h_lambda, h_lambda + (M->lv.size() > 0 ? M->lv.size() - 1 : 0) * M->n_inst);
    for (size_t l = 0; l + 1 < M->lv.size(); ++l) {
      const Level& L = *M->lv[l];
      for (int t = 0; t < L.n_act; ++t)
        BLK_REQUIRE(lam[l * M->n_inst + L.seg_inst[t]] > 0.0, BLKAMG_EINVAL, "lambda must be positive");
    }
  }
  smoother_refresh(M, h_lambda ? lam.data() : nullptr, as_stream(stream));
  BLK_API_END
}

int amg_smoother_refresh(amg_t M, const double* h_lambda, void* stream) {
  BLK_API_BEGIN
  BLK_REQUIRE(M != nullptr, BLKAMG_EINVAL, "M is NULL");
  if (h_lambda)
    for (size_t l = 0; l + 1 < M->lv.size(); ++l) {
      const Level& L = *M->lv[l];
      for (int t = 0; t < L.n_act; ++t)
        BLK_REQUIRE(h_lambda[l * M->n_inst + L.seg_inst[t]] > 0.0, BLKAMG_EINVAL, "lambda must be positive");
    }
  smoother_refresh(M, h_lambda, as_stream(stream));
  BLK_API_END
}

int amg_features(amg_t M, float* d_feat, int32_t* n_samples, int32_t* h_level, int32_t* h_inst, void* stream) {
  BLK_API_BEGIN
  BLK_REQUIRE(M != nullptr, BLKAMG_EINVAL, "M is NULL");
  if (n_samples) *n_samples = M->n_samples;
  for (size_t l = 0; l < M->lv.size(); ++l)
    for (int t = 0; t < M->lv[l]->n_act; ++t) {
      const int k = M->sample_base[l] + t;
      if (h_level) h_level[k] = static_cast<int32_t>(l);
      if (h_inst) h_inst[k] = M->lv[l]->seg_inst[t];
    }
  if (d_feat) {
    hipStream_t s = as_stream(stream);
    for (auto& lp : M->lv)
      if (lp->n_act > 0) compute_dinv(M, *lp, s);
    all_features(M, d_feat, s);
    HIP_CHECK(hipStreamSynchronize(s));
  }
  BLK_API_END
}

int amg_judge_lambdas(amg_t M, int32_t k, double* h_lam, void* stream) {
  BLK_API_BEGIN
  BLK_REQUIRE(M != nullptr && h_lam != nullptr, BLKAMG_EINVAL, "NULL argument");
  BLK_REQUIRE(k >= 2 && k <= kMaxLanczos, BLKAMG_EINVAL, "k must be in 2..64");
  hipStream_t s = as_stream(stream);
  const size_t nl = M->lv.size();
  for (size_t l = 0; l + 1 < nl; ++l) {
    for (int t = 0; t < M->n_inst; ++t) h_lam[l * M->n_inst + t] = 0.0;
    const Level& L = *M->lv[l];
    const std::vector<double> lam = judge_level(M, static_cast<int>(l), k, s);
    for (int t = 0; t < L.n_act; ++t) h_lam[l * M->n_inst + L.seg_inst[t]] = lam[t];
  }
  HIP_CHECK(hipStreamSynchronize(s));
  BLK_API_END
}

int amg_set_eig_model(amg_t M, const float* h_model, int32_t n_floats) {
  BLK_API_BEGIN
  BLK_REQUIRE(M != nullptr && h_model != nullptr, BLKAMG_EINVAL, "NULL argument");
  BLK_REQUIRE(n_floats == kMlpModel, BLKAMG_EINVAL, "a model has BLKAMG_MLP_MODEL floats");
  set_model(M, h_model);
  BLK_API_END
}

int amg_setup_weights(amg_t M, double* h_lambda, double* h_omega, int32_t* h_learned) {
  BLK_API_BEGIN
  BLK_REQUIRE(M != nullptr, BLKAMG_EINVAL, "M is NULL");
  const size_t nl = M->lv.size();
  for (size_t l = 0; l + 1 < nl; ++l) {
    if (h_learned) h_learned[l] = l < M->setup_learned.size() ? M->setup_learned[l] : 0;
    for (int t = 0; t < M->n_inst; ++t) {
      const size_t k = l * M->n_inst + t;
      if (h_lambda) h_lambda[k] = k < M->setup_lam.size() ? M->setup_lam[k] : 0.0;
      if (h_omega) h_omega[k] = k < M->setup_omega.size() ? M->setup_omega[k] : 0.0;
    }
  }
  BLK_API_END
}

int amg_eig_status(amg_t M, int32_t* h_fallback, double* h_growth, double* h_omega) {
  BLK_API_BEGIN
  BLK_REQUIRE(M != nullptr, BLKAMG_EINVAL, "M is NULL");
  const size_t nl = M->lv.size();
  for (size_t l = 0; l + 1 < nl; ++l) {
    if (h_fallback) h_fallback[l] = l < M->fallback.size() ? M->fallback[l] : 0;
    for (int t = 0; t < M->n_inst; ++t) {
      const size_t k = l * M->n_inst + t;
      if (h_growth) h_growth[k] = k < M->growth.size() ? M->growth[k] : 0.0;
      if (h_omega) h_omega[k] = k < M->omega.size() ? M->omega[k] : 0.0;
    }
  }
  BLK_API_END
}

int amg_guard_status(amg_t M, int32_t* armed, int32_t* restarts) {
  BLK_API_BEGIN
  BLK_REQUIRE(M != nullptr, BLKAMG_EINVAL, "M is NULL");
  if (armed) *armed = M->guard_armed ? 1 : 0;
  if (restarts) *restarts = M->guard_restarts;
  BLK_API_END
}

int vcycle_apply_ex(amg_t M, const void* d_r, void* d_z, int vec_dtype, int32_t nrhs, void* stream) {
  BLK_API_BEGIN
  BLK_REQUIRE(M != nullptr && d_r != nullptr && d_z != nullptr, BLKAMG_EINVAL, "NULL argument");
  BLK_REQUIRE(vec_dtype == BLKAMG_F64 || vec_dtype == BLKAMG_F32, BLKAMG_EINVAL, "vec_dtype must be F64 or F32");
  if (vec_dtype == BLKAMG_F64)
    return vcycle_apply(M, static_cast<const double*>(d_r), static_cast<double*>(d_z), nrhs, stream);
  BLK_REQUIRE(M->T == BLKAMG_F32, BLKAMG_EINVAL, "FP32 vectors need an F32 hierarchy");
  BLK_REQUIRE(nrhs == 1 || nrhs == 8, BLKAMG_EINVAL, "vcycle_apply supports nrhs 1 or 8");
  BLK_REQUIRE(d_r != d_z, BLKAMG_EINVAL, "r and z must not alias");
  hipStream_t s = as_stream(stream);
  ensure_vectors(M, nrhs);
  if (M->guard_armed) mlp_check_levels(M, s);
  const float* r = static_cast<const float*>(d_r);
  float* z = static_cast<float*>(d_z);
  if (nrhs == 1) vcycle_level<float, 1>(M, 0, r, z, s);
  else vcycle_level<float, 8>(M, 0, r, z, s);
  BLK_API_END
}

int vcycle_apply(amg_t M, const double* d_r, double* d_z, int32_t nrhs, void* stream) {
  BLK_API_BEGIN
  BLK_REQUIRE(M != nullptr && d_r != nullptr && d_z != nullptr, BLKAMG_EINVAL, "NULL argument");
  BLK_REQUIRE(nrhs == 1 || nrhs == 8, BLKAMG_EINVAL, "vcycle_apply supports nrhs 1 or 8");
  BLK_REQUIRE(d_r != d_z, BLKAMG_EINVAL, "r and z must not alias");
  ensure_vectors(M, nrhs);
  if (M->guard_armed) mlp_check_levels(M, as_stream(stream));
  vcycle(M, d_r, d_z, nrhs, as_stream(stream));
  BLK_API_END
}

int pcg_solve(bsr_t A, amg_t M, const double* d_b, double* d_x, double rtol, int32_t maxit, int32_t nrhs,
              int32_t* iters, double* relres, void* stream) {
  BLK_API_BEGIN
  BLK_REQUIRE(A != nullptr && M != nullptr && d_b != nullptr && d_x != nullptr, BLKAMG_EINVAL, "NULL argument");
  BLK_REQUIRE(nrhs == 1 || nrhs == 8, BLKAMG_EINVAL, "pcg_solve supports nrhs 1 or 8");
  BLK_REQUIRE(A->dtype == BLKAMG_F64 && A->br == A->bc && A->nbr == A->nbc, BLKAMG_EINVAL, "A must be square F64");
  BLK_REQUIRE(static_cast<int64_t>(A->nbr) * A->br == static_cast<int64_t>(M->lv[0]->n), BLKAMG_EINVAL,
              "A and the hierarchy have different sizes");
  BLK_REQUIRE(A->br == 3 || A->br == 6, BLKAMG_EINVAL, "A must have 3x3 or 6x6 blocks");
  BLK_REQUIRE(maxit >= 0 && rtol >= 0.0, BLKAMG_EINVAL, "bad rtol or maxit");
  hipStream_t s = as_stream(stream);
  if (M->n_inst == 1 && nrhs == 1) return pcg_single(A, M, d_b, d_x, rtol, maxit, iters, relres, s);
  if (M->guard_armed) mlp_check_levels(M, s);
  if (nrhs == 1) return pcg_batched<1>(A, M, d_b, d_x, rtol, maxit, iters, relres, s);
  return pcg_batched<8>(A, M, d_b, d_x, rtol, maxit, iters, relres, s);
  BLK_API_END
}

}  // extern "C"

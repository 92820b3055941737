// Host-side smoothed-aggregation setup (cold path): greedy aggregation over the
// block graph (paper §2.2, §3.2), rigid-body near-null space and the tentative
// prolongator by per-aggregate QR (paper §2.2, §2.3).  Integer-only aggregation so
// that it is reproducible bit for bit.
#include "sa_host.hpp"

#include <algorithm>
#include <cmath>
#include <memory>
#include <string>

#include "common.hpp"
#include "internal.hpp"

namespace blk {

int32_t aggregate_host(int32_t nbr, const int32_t* rowptr, const int32_t* colidx, const uint8_t* dirichlet,
                       const uint8_t* strong, std::vector<int32_t>& agg) {
  auto is_dir = [&](int32_t i) { return dirichlet != nullptr && dirichlet[i] != 0; };
  auto is_nbr = [&](int32_t i, int32_t k) {
    const int32_t j = colidx[k];
    return j != i && !is_dir(j) && (strong == nullptr || strong[k] != 0);
  };
  agg.assign(static_cast<size_t>(nbr), -1);
  int32_t n_agg = 0;
  // phase 1: roots in natural order whose whole neighbourhood is still free
  for (int32_t i = 0; i < nbr; ++i) {
    if (is_dir(i) || agg[i] >= 0) continue;
    bool free = true;
    for (int32_t k = rowptr[i]; k < rowptr[i + 1] && free; ++k)
      if (is_nbr(i, k) && agg[colidx[k]] >= 0) free = false;
    if (!free) continue;
    agg[i] = n_agg;
    for (int32_t k = rowptr[i]; k < rowptr[i + 1]; ++k)
      if (is_nbr(i, k)) agg[colidx[k]] = n_agg;
    ++n_agg;
  }
  // phase 2: leftovers join the phase-1 aggregate with most neighbours (ties: smallest id)
  const std::vector<int32_t> phase1 = agg;
  std::vector<std::pair<int32_t, int32_t>> cnt;
  for (int32_t i = 0; i < nbr; ++i) {
    if (is_dir(i) || phase1[i] >= 0) continue;
    cnt.clear();
    for (int32_t k = rowptr[i]; k < rowptr[i + 1]; ++k) {
      if (!is_nbr(i, k)) continue;
      const int32_t g = phase1[colidx[k]];
      if (g < 0) continue;
      bool hit = false;
      for (auto& c : cnt)
        if (c.first == g) { c.second++; hit = true; break; }
      if (!hit) cnt.emplace_back(g, 1);
    }
    if (cnt.empty()) {
      agg[i] = n_agg++;
      continue;
    }
    int32_t best = -1, best_c = -1;
    for (const auto& c : cnt)
      if (c.second > best_c || (c.second == best_c && c.first < best)) { best = c.first; best_c = c.second; }
    agg[i] = best;
  }
  return n_agg;
}

std::vector<double> rigid_body_modes(int32_t nbr, const double* coords) {
  std::vector<double> B(static_cast<size_t>(nbr) * 18, 0.0);
  for (int32_t i = 0; i < nbr; ++i) {
    const double x = coords[3 * i], y = coords[3 * i + 1], z = coords[3 * i + 2];
    double* b = &B[static_cast<size_t>(i) * 18];  // rows c = 0..2, columns 0..5
    b[0 * 6 + 0] = 1.0;
    b[1 * 6 + 1] = 1.0;
    b[2 * 6 + 2] = 1.0;
    b[0 * 6 + 3] = -y;  // rotation about z
    b[1 * 6 + 3] = x;
    b[1 * 6 + 4] = -z;  // rotation about x
    b[2 * 6 + 4] = y;
    b[0 * 6 + 5] = z;   // rotation about y
    b[2 * 6 + 5] = -x;
  }
  return B;
}

namespace {

// Thin QR of the column-major m x nc matrix M by Householder reflections; on exit
// Q (m x nc, column-major) and R (nc x nc, row-major) with diag(R) > 0.
bool householder_qr(int m, int nc, std::vector<double>& M, std::vector<double>& Q, std::vector<double>& R,
                    double tol) {
  std::vector<double> V(static_cast<size_t>(m) * nc, 0.0), beta(nc, 0.0);
  double scale = 0.0;
  for (double v : M) scale = std::max(scale, std::fabs(v));
  for (int k = 0; k < nc; ++k) {
    double* col = &M[static_cast<size_t>(k) * m];
    double nrm2 = 0.0;
    for (int i = k; i < m; ++i) nrm2 += col[i] * col[i];
    const double nrm = std::sqrt(nrm2);
    const double alpha = col[k] >= 0 ? -nrm : nrm;
    double* v = &V[static_cast<size_t>(k) * m];
    for (int i = k; i < m; ++i) v[i] = col[i];
    v[k] -= alpha;
    double vv = 0.0;
    for (int i = k; i < m; ++i) vv += v[i] * v[i];
    beta[k] = vv > 0 ? 2.0 / vv : 0.0;
    for (int j = k; j < nc; ++j) {
      double* cj = &M[static_cast<size_t>(j) * m];
      double d = 0.0;
      for (int i = k; i < m; ++i) d += v[i] * cj[i];
      d *= beta[k];
      for (int i = k; i < m; ++i) cj[i] -= d * v[i];
    }
  }
  R.assign(static_cast<size_t>(nc) * nc, 0.0);
  for (int r = 0; r < nc; ++r)
    for (int c = r; c < nc; ++c) R[r * nc + c] = M[static_cast<size_t>(c) * m + r];
  for (int r = 0; r < nc; ++r)
    if (!(std::fabs(R[r * nc + r]) > tol * std::max(1.0, scale))) return false;
  // Q = H_0 H_1 ... H_{nc-1} applied to the first nc columns of the identity
  Q.assign(static_cast<size_t>(m) * nc, 0.0);
  for (int c = 0; c < nc; ++c) Q[static_cast<size_t>(c) * m + c] = 1.0;
  for (int k = nc - 1; k >= 0; --k) {
    const double* v = &V[static_cast<size_t>(k) * m];
    for (int c = 0; c < nc; ++c) {
      double* qc = &Q[static_cast<size_t>(c) * m];
      double d = 0.0;
      for (int i = k; i < m; ++i) d += v[i] * qc[i];
      d *= beta[k];
      for (int i = k; i < m; ++i) qc[i] -= d * v[i];
    }
  }
  for (int r = 0; r < nc; ++r) {
    if (R[r * nc + r] < 0) {
      for (int c = 0; c < nc; ++c) R[r * nc + c] = -R[r * nc + c];
      for (int i = 0; i < m; ++i) Q[static_cast<size_t>(r) * m + i] = -Q[static_cast<size_t>(r) * m + i];
    }
  }
  return true;
}

}  // namespace

void tentative_host(int32_t nbr, int32_t bs, int32_t nc, const std::vector<int32_t>& agg, int32_t n_agg,
                    const std::vector<double>& B, std::vector<double>& Pt, std::vector<double>& Bc) {
  std::vector<int32_t> start(static_cast<size_t>(n_agg) + 1, 0), members;
  for (int32_t i = 0; i < nbr; ++i)
    if (agg[i] >= 0) start[agg[i] + 1]++;
  for (int32_t g = 0; g < n_agg; ++g) start[g + 1] += start[g];
  members.resize(start[n_agg]);
  {
    std::vector<int32_t> next(start.begin(), start.end() - 1);
    for (int32_t i = 0; i < nbr; ++i)
      if (agg[i] >= 0) members[next[agg[i]]++] = i;  // ascending node order
  }
  Pt.assign(static_cast<size_t>(nbr) * bs * nc, 0.0);
  Bc.assign(static_cast<size_t>(n_agg) * nc * nc, 0.0);
  std::vector<double> M, Q, R;
  for (int32_t g = 0; g < n_agg; ++g) {
    const int cnt = start[g + 1] - start[g];
    const int m = cnt * bs;
    BLK_REQUIRE(m >= nc, BLKAMG_EINVAL, "aggregate " + std::to_string(g) + " too small for the near-null space");
    M.assign(static_cast<size_t>(m) * nc, 0.0);
    for (int t = 0; t < cnt; ++t) {
      const int32_t i = members[start[g] + t];
      for (int r = 0; r < bs; ++r)
        for (int c = 0; c < nc; ++c)
          M[static_cast<size_t>(c) * m + t * bs + r] = B[(static_cast<size_t>(i) * bs + r) * nc + c];
    }
    BLK_REQUIRE(householder_qr(m, nc, M, Q, R, 1e-10), BLKAMG_EINVAL,
                "aggregate " + std::to_string(g) + ": near-null space rank deficient");
    for (int t = 0; t < cnt; ++t) {
      const int32_t i = members[start[g] + t];
      for (int r = 0; r < bs; ++r)
        for (int c = 0; c < nc; ++c)
          Pt[(static_cast<size_t>(i) * bs + r) * nc + c] = Q[static_cast<size_t>(c) * m + t * bs + r];
    }
    std::copy(R.begin(), R.end(), Bc.begin() + static_cast<size_t>(g) * nc * nc);
  }
}

}  // namespace blk

extern "C" int sa_aggregate(int32_t nbr, const int32_t* h_rowptr, const int32_t* h_colidx,
                            const uint8_t* h_dirichlet, int32_t* h_agg, int32_t* n_agg) {
  BLK_API_BEGIN
  BLK_REQUIRE(nbr >= 0, BLKAMG_EINVAL, "negative size");
  BLK_REQUIRE(h_rowptr != nullptr && (nbr == 0 || h_agg != nullptr) && n_agg != nullptr, BLKAMG_EINVAL,
              "NULL argument");
  BLK_REQUIRE(h_rowptr[0] == 0 && (h_rowptr[nbr] == 0 || h_colidx != nullptr), BLKAMG_EINVAL, "bad rowptr");
  for (int32_t r = 0; r < nbr; ++r) {
    BLK_REQUIRE(h_rowptr[r] <= h_rowptr[r + 1], BLKAMG_EINVAL, "rowptr not monotone");
    for (int32_t k = h_rowptr[r]; k < h_rowptr[r + 1]; ++k)
      BLK_REQUIRE(h_colidx[k] >= 0 && h_colidx[k] < nbr, BLKAMG_EINVAL, "column index out of range");
  }
  std::vector<int32_t> agg;
  *n_agg = blk::aggregate_host(nbr, h_rowptr, h_colidx, h_dirichlet, nullptr, agg);
  std::copy(agg.begin(), agg.end(), h_agg);
  BLK_API_END
}

// Host setup of one smoothed-aggregation level from a block pattern (paper §2.2):
// aggregation, tentative prolongator, coarse near-null space and the pattern of the
// smoothed prolongator.
struct sa_result_s {
  int32_t n_nodes = 0, n_agg = 0;
  std::vector<int32_t> agg;
  std::vector<int32_t> pt_rowptr, pt_colidx;  // P~: one block per aggregated row
  std::vector<double> pt_val;                 // [pt_nnzb][3][6]
  std::vector<double> bc;                     // [n_agg][6][6]
  std::vector<int32_t> sp_rowptr, sp_colidx;  // pattern of A P~
};

extern "C" int sa_setup_host(int32_t n_nodes, const int32_t* h_rowptr, const int32_t* h_colidx,
                             const uint8_t* h_dirichlet, const double* h_coords, const blkamg_opts* opts,
                             sa_result_t* out) {
  BLK_API_BEGIN
  BLK_REQUIRE(out != nullptr, BLKAMG_EINVAL, "output pointer is NULL");
  *out = nullptr;
  BLK_REQUIRE(n_nodes >= 0 && h_rowptr != nullptr, BLKAMG_EINVAL, "bad size or NULL rowptr");
  BLK_REQUIRE(n_nodes == 0 || h_coords != nullptr, BLKAMG_EINVAL, "coordinates are NULL");
  BLK_REQUIRE(h_rowptr[0] == 0 && (h_rowptr[n_nodes] == 0 || h_colidx != nullptr), BLKAMG_EINVAL, "bad rowptr");
  BLK_REQUIRE(opts == nullptr || opts->strength_eps == 0.0, BLKAMG_EINVAL,
              "a pattern-only setup has no block norms: strength_eps must be 0");
  for (int32_t r = 0; r < n_nodes; ++r) {
    BLK_REQUIRE(h_rowptr[r] <= h_rowptr[r + 1], BLKAMG_EINVAL, "rowptr not monotone");
    for (int32_t k = h_rowptr[r]; k < h_rowptr[r + 1]; ++k) {
      BLK_REQUIRE(h_colidx[k] >= 0 && h_colidx[k] < n_nodes, BLKAMG_EINVAL, "column index out of range");
      BLK_REQUIRE(k == h_rowptr[r] || h_colidx[k] > h_colidx[k - 1], BLKAMG_EINVAL,
                  "column indices must be strictly ascending per row");
    }
  }
  auto R = std::make_unique<sa_result_s>();
  R->n_nodes = n_nodes;
  R->n_agg = blk::aggregate_host(n_nodes, h_rowptr, h_colidx, h_dirichlet, nullptr, R->agg);
  constexpr int bs = 3, nc = 6;
  std::vector<double> Pt;
  blk::tentative_host(n_nodes, bs, nc, R->agg, R->n_agg, blk::rigid_body_modes(n_nodes, h_coords), Pt, R->bc);
  R->pt_rowptr.assign(static_cast<size_t>(n_nodes) + 1, 0);
  for (int32_t i = 0; i < n_nodes; ++i) {
    if (R->agg[i] >= 0) {
      R->pt_colidx.push_back(R->agg[i]);
      R->pt_val.insert(R->pt_val.end(), Pt.begin() + static_cast<size_t>(i) * bs * nc,
                       Pt.begin() + static_cast<size_t>(i + 1) * bs * nc);
    }
    R->pt_rowptr[i + 1] = static_cast<int32_t>(R->pt_colidx.size());
  }
  const std::vector<int32_t> arp(h_rowptr, h_rowptr + n_nodes + 1), aci(h_colidx, h_colidx + h_rowptr[n_nodes]);
  blk::structural_product_host(n_nodes, arp, aci, R->n_agg, R->pt_rowptr, R->pt_colidx, R->sp_rowptr, R->sp_colidx);
  *out = R.release();
  BLK_API_END
}

extern "C" int sa_result_info(sa_result_t r, int32_t* n_agg, int64_t* pt_nnzb, int64_t* sp_nnzb) {
  BLK_API_BEGIN
  BLK_REQUIRE(r != nullptr, BLKAMG_EINVAL, "result is NULL");
  if (n_agg) *n_agg = r->n_agg;
  if (pt_nnzb) *pt_nnzb = static_cast<int64_t>(r->pt_colidx.size());
  if (sp_nnzb) *sp_nnzb = static_cast<int64_t>(r->sp_colidx.size());
  BLK_API_END
}

extern "C" int sa_result_arrays(sa_result_t r, const int32_t** agg, const int32_t** pt_rowptr,
                                const int32_t** pt_colidx, const double** pt_val, const double** bc,
                                const int32_t** sp_rowptr, const int32_t** sp_colidx) {
  BLK_API_BEGIN
  BLK_REQUIRE(r != nullptr, BLKAMG_EINVAL, "result is NULL");
  if (agg) *agg = r->agg.data();
  if (pt_rowptr) *pt_rowptr = r->pt_rowptr.data();
  if (pt_colidx) *pt_colidx = r->pt_colidx.data();
  if (pt_val) *pt_val = r->pt_val.data();
  if (bc) *bc = r->bc.data();
  if (sp_rowptr) *sp_rowptr = r->sp_rowptr.data();
  if (sp_colidx) *sp_colidx = r->sp_colidx.data();
  BLK_API_END
}

extern "C" int sa_result_free(sa_result_t r) {
  BLK_API_BEGIN
  delete r;
  BLK_API_END
}

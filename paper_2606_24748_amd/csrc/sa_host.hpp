// Host-side smoothed-aggregation setup pieces (cold path, paper §2.2, §3.2).
#pragma once

#include <cstdint>
#include <vector>

namespace blk {

// Greedy aggregation over the block graph.  `strong` (optional, one flag per stored
// block) removes weak couplings; Dirichlet rows are excluded.  Returns n_agg.
int32_t aggregate_host(int32_t nbr, const int32_t* rowptr, const int32_t* colidx, const uint8_t* dirichlet,
                       const uint8_t* strong, std::vector<int32_t>& agg);

// Six rigid-body modes per node from coordinates: [nbr][3][6].
std::vector<double> rigid_body_modes(int32_t nbr, const double* coords);

// Tentative prolongator: per aggregate, thin Householder QR of the stacked
// near-null-space rows (members ascending), signs fixed so that diag(R) > 0.
// B: [nbr][bs][nc]; outputs Pt: [nbr][bs][nc] (zero for unaggregated rows) and
// Bc: [n_agg][nc][nc].  Throws EINVAL when an aggregate is rank deficient.
void tentative_host(int32_t nbr, int32_t bs, int32_t nc, const std::vector<int32_t>& agg, int32_t n_agg,
                    const std::vector<double>& B, std::vector<double>& Pt, std::vector<double>& Bc);

}  // namespace blk

// Distance-2 aggregation on the device by Luby rounds (paper §6: the device MIS
// coarsener with deterministic hash priorities).
//
// The graph is the block pattern of A without the diagonal and without Dirichlet
// vertices.  Vertex i has the priority key_i = (high 32 bits of splitmix64(seed ^ i))
// above (i + 1), so keys are distinct and positive.  One round is four passes over
// the pattern, one thread per vertex:
//   1. m1_i = largest key of an undecided vertex in {i} and its neighbours;
//   2. an undecided i whose key equals the largest m1 over {i} and its neighbours
//      (the largest undecided key within distance 2) becomes a root;
//   3. near_i = some vertex of {i} and its neighbours became a root this round;
//   4. an undecided i with near set on itself or a neighbour (within distance 2 of a
//      new root) is decided; the undecided vertices left are counted.
// The host reads the count after each round (every round decides at least the
// vertex with the largest undecided key, so the loop ends).  Roots are then numbered
// in vertex order by a prefix sum; neighbours of a root join it (roots are at least
// three apart, so that root is unique) and the remaining vertices join the
// neighbouring aggregate holding most of their neighbours, ties to the smallest id.
#include <algorithm>

#include <hipcub/hipcub.hpp>

#include "internal.hpp"

namespace blk {
namespace {

// splitmix64 output function (Steele, Lea and Flood 2014) applied to one state
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

enum : uint8_t { kUndecided = 0, kRoot = 1, kOut = 2, kNewRoot = 3 };

__device__ __forceinline__ bool free_vertex(const uint8_t* __restrict__ dir, int32_t v) {
  return dir == nullptr || dir[v] == 0;
}

__global__ void mis_init_kernel(int32_t n, const uint8_t* __restrict__ dir, uint64_t seed, uint64_t* __restrict__ key,
                                uint8_t* __restrict__ state) {
  const int32_t i = static_cast<int32_t>(blockIdx.x * blockDim.x + threadIdx.x);
  if (i >= n) return;
  const uint64_t h = mix64(seed ^ static_cast<uint64_t>(i));
  key[i] = ((h >> 32) << 32) | static_cast<uint64_t>(i + 1);
  state[i] = free_vertex(dir, i) ? kUndecided : kOut;
}

// pass 1: largest undecided key among {i} and its neighbours
__global__ void mis_max1_kernel(int32_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                const uint8_t* __restrict__ dir, const uint64_t* __restrict__ key,
                                const uint8_t* __restrict__ state, uint64_t* __restrict__ m1) {
  const int32_t i = static_cast<int32_t>(blockIdx.x * blockDim.x + threadIdx.x);
  if (i >= n) return;
  uint64_t m = 0;
  if (free_vertex(dir, i)) {
    if (state[i] == kUndecided) m = key[i];
    for (int32_t t = rp[i]; t < rp[i + 1]; ++t) {
      const int32_t j = ci[t];
      if (j != i && free_vertex(dir, j) && state[j] == kUndecided) m = key[j] > m ? key[j] : m;
    }
  }
  m1[i] = m;
}

// pass 2: an undecided vertex holding the largest undecided key within distance 2 becomes a root
__global__ void mis_select_kernel(int32_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                  const uint8_t* __restrict__ dir, const uint64_t* __restrict__ key,
                                  const uint64_t* __restrict__ m1, uint8_t* __restrict__ state) {
  const int32_t i = static_cast<int32_t>(blockIdx.x * blockDim.x + threadIdx.x);
  if (i >= n || state[i] != kUndecided) return;
  uint64_t m = m1[i];
  for (int32_t t = rp[i]; t < rp[i + 1]; ++t) {
    const int32_t j = ci[t];
    if (j != i && free_vertex(dir, j)) m = m1[j] > m ? m1[j] : m;
  }
  if (m == key[i]) state[i] = kNewRoot;
}

// pass 3: a new root among {i} and its neighbours
__global__ void mis_near_kernel(int32_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                const uint8_t* __restrict__ dir, const uint8_t* __restrict__ state,
                                uint8_t* __restrict__ near) {
  const int32_t i = static_cast<int32_t>(blockIdx.x * blockDim.x + threadIdx.x);
  if (i >= n) return;
  uint8_t f = 0;
  if (free_vertex(dir, i)) {
    f = state[i] == kNewRoot;
    for (int32_t t = rp[i]; t < rp[i + 1] && !f; ++t) {
      const int32_t j = ci[t];
      if (j != i && free_vertex(dir, j) && state[j] == kNewRoot) f = 1;
    }
  }
  near[i] = f;
}

// pass 4: decide the undecided vertices within distance 2 of a new root, promote the
// new roots, count what stays undecided
__global__ void mis_decide_kernel(int32_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                  const uint8_t* __restrict__ dir, const uint8_t* __restrict__ near,
                                  uint8_t* __restrict__ state, int32_t* __restrict__ n_undecided) {
  const int32_t i = static_cast<int32_t>(blockIdx.x * blockDim.x + threadIdx.x);
  if (i >= n) return;
  const uint8_t s = state[i];
  if (s == kNewRoot) {
    state[i] = kRoot;
  } else if (s == kUndecided) {
    bool hit = near[i] != 0;
    for (int32_t t = rp[i]; t < rp[i + 1] && !hit; ++t) {
      const int32_t j = ci[t];
      if (j != i && free_vertex(dir, j) && near[j]) hit = true;
    }
    if (hit) state[i] = kOut;
    else atomicAdd(n_undecided, 1);
  }
}

__global__ void mis_zero_kernel(int32_t* __restrict__ c) {
  if (threadIdx.x == 0) c[0] = 0;
}

__global__ void mis_root_flag_kernel(int32_t n, const uint8_t* __restrict__ state, int32_t* __restrict__ flag) {
  const int32_t i = static_cast<int32_t>(blockIdx.x * blockDim.x + threadIdx.x);
  if (i < n) flag[i] = state[i] == kRoot;
}

// phase 1: roots take their number, neighbours of a root join it, others wait (-2)
__global__ void mis_phase1_kernel(int32_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                  const uint8_t* __restrict__ dir, const uint8_t* __restrict__ state,
                                  const int32_t* __restrict__ root_id, int32_t* __restrict__ agg1) {
  const int32_t i = static_cast<int32_t>(blockIdx.x * blockDim.x + threadIdx.x);
  if (i >= n) return;
  int32_t g = -1;
  if (free_vertex(dir, i)) {
    if (state[i] == kRoot) {
      g = root_id[i];
    } else {
      g = -2;
      for (int32_t t = rp[i]; t < rp[i + 1]; ++t) {
        const int32_t j = ci[t];
        if (j != i && free_vertex(dir, j) && state[j] == kRoot) {
          g = root_id[j];
          break;
        }
      }
    }
  }
  agg1[i] = g;
}

// phase 2: a waiting vertex joins the phase-1 aggregate holding most of its neighbours
__global__ void mis_phase2_kernel(int32_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                  const uint8_t* __restrict__ dir, const int32_t* __restrict__ agg1,
                                  int32_t* __restrict__ agg) {
  const int32_t i = static_cast<int32_t>(blockIdx.x * blockDim.x + threadIdx.x);
  if (i >= n) return;
  int32_t g = agg1[i];
  if (g == -2) {
    int32_t best = -1, best_c = 0;
    const int32_t t0 = rp[i], t1 = rp[i + 1];
    for (int32_t t = t0; t < t1; ++t) {
      const int32_t j = ci[t];
      if (j == i || !free_vertex(dir, j)) continue;
      const int32_t h = agg1[j];
      if (h < 0) continue;
      int32_t c = 0;
      for (int32_t u = t0; u < t1; ++u) {
        const int32_t k = ci[u];
        if (k != i && free_vertex(dir, k) && agg1[k] == h) ++c;
      }
      if (c > best_c || (c == best_c && h < best)) {
        best = h;
        best_c = c;
      }
    }
    g = best;  // every waiting vertex neighbours a phase-1 vertex (maximality)
  }
  agg[i] = g;
}

}  // namespace
}  // namespace blk

using namespace blk;

extern "C" {

int sa_aggregate_device(bsr_t A, const uint8_t* d_dirichlet, uint64_t seed, int32_t* d_agg, int32_t* n_agg,
                        int32_t* n_rounds, void* stream) {
  BLK_API_BEGIN
  BLK_REQUIRE(A != nullptr && n_agg != nullptr, BLKAMG_EINVAL, "NULL argument");
  BLK_REQUIRE(A->nbr == A->nbc, BLKAMG_EINVAL, "A must be square");
  BLK_REQUIRE(A->nbr == 0 || d_agg != nullptr, BLKAMG_EINVAL, "d_agg is NULL");
  const int32_t n = A->nbr;
  *n_agg = 0;
  if (n_rounds) *n_rounds = 0;
  if (n == 0) return BLKAMG_OK;
  hipStream_t s = as_stream(stream);
  DevBuf<uint64_t> key(static_cast<size_t>(n)), m1(static_cast<size_t>(n));
  DevBuf<uint8_t> state(static_cast<size_t>(n)), near(static_cast<size_t>(n));
  DevBuf<int32_t> flag(static_cast<size_t>(n)), root_id(static_cast<size_t>(n)), agg1(static_cast<size_t>(n));
  DevBuf<int32_t> counter(1);
  const int grid = (n + 255) / 256;
  mis_init_kernel<<<grid, 256, 0, s>>>(n, d_dirichlet, seed, key.p, state.p);
  HIP_CHECK(hipGetLastError());
  int32_t rounds = 0, left = n;
  while (left > 0) {
    BLK_REQUIRE(rounds < n, BLKAMG_EINVAL, "aggregation rounds did not finish");
    ++rounds;
    mis_max1_kernel<<<grid, 256, 0, s>>>(n, A->rowptr, A->colidx, d_dirichlet, key.p, state.p, m1.p);
    mis_select_kernel<<<grid, 256, 0, s>>>(n, A->rowptr, A->colidx, d_dirichlet, key.p, m1.p, state.p);
    mis_near_kernel<<<grid, 256, 0, s>>>(n, A->rowptr, A->colidx, d_dirichlet, state.p, near.p);
    mis_zero_kernel<<<1, 64, 0, s>>>(counter.p);
    mis_decide_kernel<<<grid, 256, 0, s>>>(n, A->rowptr, A->colidx, d_dirichlet, near.p, state.p, counter.p);
    HIP_CHECK(hipGetLastError());
    HIP_CHECK(hipMemcpyAsync(&left, counter.p, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIP_CHECK(hipStreamSynchronize(s));
  }
  mis_root_flag_kernel<<<grid, 256, 0, s>>>(n, state.p, flag.p);
  HIP_CHECK(hipGetLastError());
  size_t tmp_bytes = 0;
  HIP_CHECK(hipcub::DeviceScan::ExclusiveSum(nullptr, tmp_bytes, flag.p, root_id.p, n, s));
  DevBuf<char> tmp(std::max<size_t>(tmp_bytes, 1));
  HIP_CHECK(hipcub::DeviceScan::ExclusiveSum(tmp.p, tmp_bytes, flag.p, root_id.p, n, s));
  mis_phase1_kernel<<<grid, 256, 0, s>>>(n, A->rowptr, A->colidx, d_dirichlet, state.p, root_id.p, agg1.p);
  mis_phase2_kernel<<<grid, 256, 0, s>>>(n, A->rowptr, A->colidx, d_dirichlet, agg1.p, d_agg);
  HIP_CHECK(hipGetLastError());
  int32_t last_id = 0, last_flag = 0;
  HIP_CHECK(hipMemcpyAsync(&last_id, root_id.p + (n - 1), sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIP_CHECK(hipMemcpyAsync(&last_flag, flag.p + (n - 1), sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIP_CHECK(hipStreamSynchronize(s));
  *n_agg = last_id + last_flag;
  if (n_rounds) *n_rounds = rounds;
  BLK_API_END
}

}  // extern "C"

// Distance-2 aggregation on the device by Luby rounds (paper §6: the device MIS
// coarsener with deterministic hash priorities).
//
// The graph is the block pattern of A without the diagonal and without Dirichlet
// vertices.  Vertex i has the priority key_i = (high 32 bits of splitmix64(seed ^ i))
// above (i + 1), so keys are distinct and positive.  One round is four passes over
// the pattern (a group of lanes per vertex):
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
#include <mutex>
#include <string>

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

// priorities and states; the free (undecided) vertices are counted per workgroup in
// LDS, then with one global atomic per workgroup
__global__ __launch_bounds__(256) void mis_init_kernel(int32_t n, const uint8_t* __restrict__ dir, uint64_t seed,
                                                       uint64_t* __restrict__ key, uint8_t* __restrict__ state,
                                                       int32_t* __restrict__ n_undecided) {
  __shared__ int32_t block_free;
  if (threadIdx.x == 0) block_free = 0;
  __syncthreads();
  const int32_t i = static_cast<int32_t>(blockIdx.x * blockDim.x + threadIdx.x);
  if (i < n) {
    const uint64_t h = mix64(seed ^ static_cast<uint64_t>(i));
    key[i] = ((h >> 32) << 32) | static_cast<uint64_t>(i + 1);
    const bool f = free_vertex(dir, i);
    state[i] = f ? kUndecided : kOut;
    if (f) atomicAdd(&block_free, 1);
  }
  __syncthreads();
  if (threadIdx.x == 0 && block_free > 0) atomicAdd(n_undecided, block_free);
}

// The passes over the graph give each vertex a group of kG lanes that stride over its
// neighbours (consecutive lanes read consecutive column indices) and combine their
// findings by shuffles; lane 0 of the group writes the vertex's result.  Eight lanes
// (27 neighbours: four trips) keep the number of waves, which bounds these light
// passes, at a quarter of what 32 lanes would launch.
constexpr int kG = 8;

__device__ __forceinline__ uint64_t group_max(uint64_t v) {
#pragma unroll
  for (int off = kG / 2; off > 0; off >>= 1) {
    const uint64_t o = __shfl_xor(v, off, kG);
    v = o > v ? o : v;
  }
  return v;
}

struct GroupRow {
  int32_t i, lane;
  bool active;
};

__device__ __forceinline__ GroupRow group_row(int32_t n) {
  const int64_t g = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  GroupRow r;
  r.i = static_cast<int32_t>(g / kG);
  r.lane = static_cast<int32_t>(g % kG);
  r.active = r.i < n;
  return r;
}

// pass 1: largest undecided key among {i} and its neighbours
__global__ void mis_max1_kernel(int32_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                const uint8_t* __restrict__ dir, const uint64_t* __restrict__ key,
                                const uint8_t* __restrict__ state, uint64_t* __restrict__ m1) {
  const GroupRow r = group_row(n);
  const bool use = r.active && free_vertex(dir, r.i);
  uint64_t m = 0;
  if (use) {
    if (r.lane == 0 && state[r.i] == kUndecided) m = key[r.i];
    for (int32_t t = rp[r.i] + r.lane; t < rp[r.i + 1]; t += kG) {
      const int32_t j = ci[t];
      if (j != r.i && free_vertex(dir, j) && state[j] == kUndecided) m = key[j] > m ? key[j] : m;
    }
  }
  m = group_max(m);
  if (r.active && r.lane == 0) m1[r.i] = m;
}

// pass 2: an undecided vertex holding the largest undecided key within distance 2 becomes a root
__global__ void mis_select_kernel(int32_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                  const uint8_t* __restrict__ dir, const uint64_t* __restrict__ key,
                                  const uint64_t* __restrict__ m1, uint8_t* __restrict__ state) {
  const GroupRow r = group_row(n);
  const bool use = r.active && state[r.i] == kUndecided;
  uint64_t m = 0;
  if (use) {
    if (r.lane == 0) m = m1[r.i];
    for (int32_t t = rp[r.i] + r.lane; t < rp[r.i + 1]; t += kG) {
      const int32_t j = ci[t];
      if (j != r.i && free_vertex(dir, j)) m = m1[j] > m ? m1[j] : m;
    }
  }
  m = group_max(m);
  if (use && r.lane == 0 && m == key[r.i]) state[r.i] = kNewRoot;
}

// pass 3: a new root among {i} and its neighbours
__global__ void mis_near_kernel(int32_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                const uint8_t* __restrict__ dir, const uint8_t* __restrict__ state,
                                uint8_t* __restrict__ near) {
  const GroupRow r = group_row(n);
  const bool use = r.active && free_vertex(dir, r.i);
  uint64_t f = 0;
  if (use) {
    if (r.lane == 0) f = state[r.i] == kNewRoot;
    for (int32_t t = rp[r.i] + r.lane; t < rp[r.i + 1]; t += kG) {
      const int32_t j = ci[t];
      if (j != r.i && free_vertex(dir, j) && state[j] == kNewRoot) f = 1;
    }
  }
  f = group_max(f);
  if (r.active && r.lane == 0) near[r.i] = static_cast<uint8_t>(f);
}

// pass 4: decide the undecided vertices within distance 2 of a new root, promote the
// new roots, count what stays undecided (summed per workgroup in LDS, then one global
// atomic per workgroup)
__global__ __launch_bounds__(256) void mis_decide_kernel(int32_t n, const int32_t* __restrict__ rp,
                                                         const int32_t* __restrict__ ci,
                                                         const uint8_t* __restrict__ dir,
                                                         const uint8_t* __restrict__ near, uint8_t* __restrict__ state,
                                                         int32_t* __restrict__ n_undecided) {
  __shared__ int32_t block_left;
  if (threadIdx.x == 0) block_left = 0;
  __syncthreads();
  const GroupRow r = group_row(n);
  const uint8_t s = r.active ? state[r.i] : kOut;
  uint64_t hit = 0;
  if (s == kUndecided) {
    if (r.lane == 0) hit = near[r.i] != 0;
    for (int32_t t = rp[r.i] + r.lane; t < rp[r.i + 1]; t += kG) {
      const int32_t j = ci[t];
      if (j != r.i && free_vertex(dir, j) && near[j]) hit = 1;
    }
  }
  hit = group_max(hit);
  if (r.lane == 0) {
    if (s == kNewRoot) {
      state[r.i] = kRoot;
    } else if (s == kUndecided) {
      if (hit) state[r.i] = kOut;
      else atomicAdd(&block_left, 1);
    }
  }
  __syncthreads();
  if (threadIdx.x == 0 && block_left > 0) atomicAdd(n_undecided, block_left);
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
  const GroupRow r = group_row(n);
  const bool use = r.active && free_vertex(dir, r.i) && state[r.i] != kRoot;
  uint64_t g = 0;  // root id + 1 of the (unique) neighbouring root, 0 if none
  if (use) {
    for (int32_t t = rp[r.i] + r.lane; t < rp[r.i + 1]; t += kG) {
      const int32_t j = ci[t];
      if (j != r.i && free_vertex(dir, j) && state[j] == kRoot) g = static_cast<uint64_t>(root_id[j]) + 1;
    }
  }
  g = group_max(g);
  if (!r.active || r.lane != 0) return;
  if (!free_vertex(dir, r.i)) agg1[r.i] = -1;
  else if (state[r.i] == kRoot) agg1[r.i] = root_id[r.i];
  else agg1[r.i] = g ? static_cast<int32_t>(g - 1) : -2;
}

// phase 2: a waiting vertex joins the phase-1 aggregate holding most of its neighbours
// (ties: smallest id).  Lane l holds the labels of neighbours l, l + kG, ...; each
// label's count is taken by broadcasting every neighbour label through the group, and
// (count, -label) is maximised as one 64-bit key.
__device__ __forceinline__ int32_t neighbour_label(const int32_t* __restrict__ ci, const uint8_t* __restrict__ dir,
                                                   const int32_t* __restrict__ agg1, int32_t i, int32_t t,
                                                   int32_t t1) {
  if (t >= t1) return -1;
  const int32_t j = ci[t];
  return (j != i && free_vertex(dir, j)) ? agg1[j] : -1;
}

__global__ void mis_phase2_kernel(int32_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                  const uint8_t* __restrict__ dir, const int32_t* __restrict__ agg1,
                                  int32_t* __restrict__ agg) {
  const GroupRow r = group_row(n);
  const int32_t g1 = r.active ? agg1[r.i] : -1;
  uint64_t best = 0;
  if (g1 == -2) {  // the same for every lane of the group
    const int32_t t0 = rp[r.i], t1 = rp[r.i + 1];
    for (int32_t c = t0; c < t1; c += kG) {
      const int32_t h = neighbour_label(ci, dir, agg1, r.i, c + r.lane, t1);
      uint32_t cnt = 0;
      for (int32_t c2 = t0; c2 < t1; c2 += kG) {
        const int32_t h2 = neighbour_label(ci, dir, agg1, r.i, c2 + r.lane, t1);
        for (int src = 0; src < kG; ++src) {
          // every lane takes part in the shuffle (a lane that skipped it would not
          // provide its label to the others)
          const int32_t o = __shfl(h2, src, kG);
          cnt += (h >= 0 && o == h) ? 1u : 0u;
        }
      }
      if (h >= 0) {
        const uint64_t k = (static_cast<uint64_t>(cnt) << 32) | (0xFFFFFFFFull - static_cast<uint32_t>(h));
        best = k > best ? k : best;
      }
    }
  }
  best = group_max(best);
  if (!r.active || r.lane != 0) return;
  if (g1 != -2) agg[r.i] = g1;
  else agg[r.i] = best ? static_cast<int32_t>(0xFFFFFFFFull - (best & 0xFFFFFFFFull)) : -1;
}

// Byte layout of the scratch one aggregation needs (256-byte aligned pieces).
struct MisScratch {
  size_t off[9];
  size_t total;
  size_t scan_bytes;
};

inline size_t up256(size_t b) { return (b + 255) & ~static_cast<size_t>(255); }

MisScratch mis_scratch_layout(int32_t n, hipStream_t s) {
  MisScratch L{};
  const size_t nn = static_cast<size_t>(n);
  HIP_CHECK(hipcub::DeviceScan::ExclusiveSum(nullptr, L.scan_bytes, static_cast<int32_t*>(nullptr),
                                             static_cast<int32_t*>(nullptr), n, s));
  // key, m1, state, near, flag, root_id, agg1, counter, scan temporary
  const size_t sizes[] = {nn * 8, nn * 8, nn, nn, nn * 4, nn * 4, nn * 4, 4, std::max<size_t>(L.scan_bytes, 1)};
  size_t cur = 0;
  for (int k = 0; k < 9; ++k) {
    L.off[k] = cur;
    cur += up256(sizes[k]);
  }
  L.total = cur;
  return L;
}

// The aggregation itself on caller-provided scratch of the layout above.  Every
// scratch array is written before it is read (the counter by mis_zero_kernel), so its
// previous contents do not matter.
void mis_aggregate(const bsr_s* A, const uint8_t* d_dirichlet, uint64_t seed, int32_t* d_agg, int32_t* n_agg,
                   int32_t* n_rounds, char* base, const MisScratch& L, hipStream_t s) {
  const int32_t n = A->nbr;
  auto* key = reinterpret_cast<uint64_t*>(base + L.off[0]);
  auto* m1 = reinterpret_cast<uint64_t*>(base + L.off[1]);
  auto* state = reinterpret_cast<uint8_t*>(base + L.off[2]);
  auto* near = reinterpret_cast<uint8_t*>(base + L.off[3]);
  auto* flag = reinterpret_cast<int32_t*>(base + L.off[4]);
  auto* root_id = reinterpret_cast<int32_t*>(base + L.off[5]);
  auto* agg1 = reinterpret_cast<int32_t*>(base + L.off[6]);
  auto* counter = reinterpret_cast<int32_t*>(base + L.off[7]);
  void* scan_tmp = base + L.off[8];
  size_t scan_bytes = L.scan_bytes;
  const int grid = (n + 255) / 256;
  const int64_t ggrid64 = (static_cast<int64_t>(n) * kG + 255) / 256;
  BLK_REQUIRE(ggrid64 <= INT32_MAX, BLKAMG_EINVAL, "too many vertices");
  const int ggrid = static_cast<int>(ggrid64);
  mis_zero_kernel<<<1, 64, 0, s>>>(counter);
  mis_init_kernel<<<grid, 256, 0, s>>>(n, d_dirichlet, seed, key, state, counter);
  HIP_CHECK(hipGetLastError());
  int32_t rounds = 0, left = 0;
  HIP_CHECK(hipMemcpyAsync(&left, counter, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIP_CHECK(hipStreamSynchronize(s));
  while (left > 0) {
    BLK_REQUIRE(rounds < n, BLKAMG_EINVAL, "aggregation rounds did not finish");
    ++rounds;
    mis_max1_kernel<<<ggrid, 256, 0, s>>>(n, A->rowptr, A->colidx, d_dirichlet, key, state, m1);
    mis_select_kernel<<<ggrid, 256, 0, s>>>(n, A->rowptr, A->colidx, d_dirichlet, key, m1, state);
    mis_near_kernel<<<ggrid, 256, 0, s>>>(n, A->rowptr, A->colidx, d_dirichlet, state, near);
    mis_zero_kernel<<<1, 64, 0, s>>>(counter);
    mis_decide_kernel<<<ggrid, 256, 0, s>>>(n, A->rowptr, A->colidx, d_dirichlet, near, state, counter);
    HIP_CHECK(hipGetLastError());
    HIP_CHECK(hipMemcpyAsync(&left, counter, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIP_CHECK(hipStreamSynchronize(s));
  }
  mis_root_flag_kernel<<<grid, 256, 0, s>>>(n, state, flag);
  HIP_CHECK(hipGetLastError());
  HIP_CHECK(hipcub::DeviceScan::ExclusiveSum(scan_tmp, scan_bytes, flag, root_id, n, s));
  mis_phase1_kernel<<<ggrid, 256, 0, s>>>(n, A->rowptr, A->colidx, d_dirichlet, state, root_id, agg1);
  mis_phase2_kernel<<<ggrid, 256, 0, s>>>(n, A->rowptr, A->colidx, d_dirichlet, agg1, d_agg);
  HIP_CHECK(hipGetLastError());
  int32_t last_id = 0, last_flag = 0;
  HIP_CHECK(hipMemcpyAsync(&last_id, root_id + (n - 1), sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIP_CHECK(hipMemcpyAsync(&last_flag, flag + (n - 1), sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIP_CHECK(hipStreamSynchronize(s));
  *n_agg = last_id + last_flag;
  if (n_rounds) *n_rounds = rounds;
}

// Static scratch of the allocation-free entry point: one array per GPU, loaded with
// the library's code object and held until the process ends.  Host code never
// passes the array's name to a kernel (on the host it is only a stand-in for the
// device symbol): it uses the device address that hipGetSymbolAddress returns for
// the current device, looked up once per device.
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
static __device__ __align__(256) char scratch[kNoAllocScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
char* g_scratch_ptr[kMaxDevices] = {};

char* scratch_on_current_device() {
  int dev = -1;
  HIP_CHECK(hipGetDevice(&dev));
  BLK_REQUIRE(dev >= 0 && dev < kMaxDevices, BLKAMG_EINVAL, "device ordinal out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    HIP_CHECK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    BLK_REQUIRE(p != nullptr, BLKAMG_EHIP, "hipGetSymbolAddress returned no address for the static scratch");
    g_scratch_ptr[dev] = static_cast<char*>(p);
  }
  return g_scratch_ptr[dev];
}

}  // namespace
}  // namespace blk

using namespace blk;

extern "C" {

int sa_aggregate_device_noalloc(bsr_t A, const uint8_t* d_dirichlet, uint64_t seed, int32_t* d_agg, int32_t* n_agg,
                                int32_t* n_rounds, void* stream) {
  BLK_API_BEGIN
  BLK_REQUIRE(A != nullptr && n_agg != nullptr, BLKAMG_EINVAL, "NULL argument");
  BLK_REQUIRE(A->nbr == A->nbc, BLKAMG_EINVAL, "A must be square");
  BLK_REQUIRE(A->nbr == 0 || d_agg != nullptr, BLKAMG_EINVAL, "d_agg is NULL");
  *n_agg = 0;
  if (n_rounds) *n_rounds = 0;
  if (A->nbr == 0) return BLKAMG_OK;
  hipStream_t s = as_stream(stream);
  const MisScratch L = mis_scratch_layout(A->nbr, s);
  BLK_REQUIRE(L.total <= kNoAllocScratchBytes, BLKAMG_EINVAL,
              "graph too large for the static scratch: " + std::to_string(A->nbr) + " vertices need " +
                  std::to_string(L.total) + " bytes, the limit is " + std::to_string(kNoAllocScratchBytes) +
                  " (about 2.2 million vertices); use sa_aggregate_device");
  mis_aggregate(A, d_dirichlet, seed, d_agg, n_agg, n_rounds, scratch_on_current_device(), L, s);
  BLK_API_END
}

int sa_aggregate_device(bsr_t A, const uint8_t* d_dirichlet, uint64_t seed, int32_t* d_agg, int32_t* n_agg,
                        int32_t* n_rounds, void* stream) {
  BLK_API_BEGIN
  BLK_REQUIRE(A != nullptr && n_agg != nullptr, BLKAMG_EINVAL, "NULL argument");
  BLK_REQUIRE(A->nbr == A->nbc, BLKAMG_EINVAL, "A must be square");
  BLK_REQUIRE(A->nbr == 0 || d_agg != nullptr, BLKAMG_EINVAL, "d_agg is NULL");
  *n_agg = 0;
  if (n_rounds) *n_rounds = 0;
  if (A->nbr == 0) return BLKAMG_OK;
  hipStream_t s = as_stream(stream);
  const MisScratch L = mis_scratch_layout(A->nbr, s);
  DevBuf<char> buf(L.total);  // one scratch allocation, carved into the arrays
  mis_aggregate(A, d_dirichlet, seed, d_agg, n_agg, n_rounds, buf.p, L, s);
  BLK_API_END
}

}  // extern "C"

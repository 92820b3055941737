// Shared internals of libblkamg: error handling across the C ABI, device buffers,
// value-type helpers, launch geometry for gfx950 and wavefront reductions.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <utility>
#include <vector>

#include "../../include/blkamg.h"

namespace blk {

// ---------------------------------------------------------------------------
// Errors: internal code throws Error; every exported function catches at the
// boundary, records the message and returns the status code.
// ---------------------------------------------------------------------------
struct Error {
  int code;
  std::string msg;
};

[[noreturn]] inline void fail(int code, const std::string& msg) { throw Error{code, msg}; }

void set_last_error(const std::string& msg);

#define BLK_REQUIRE(cond, code, msg)                      \
  do {                                                    \
    if (!(cond)) ::blk::fail((code), std::string(msg));   \
  } while (0)

#define HIP_CHECK(expr)                                                                  \
  do {                                                                                   \
    hipError_t e_ = (expr);                                                              \
    if (e_ != hipSuccess)                                                                \
      ::blk::fail(e_ == hipErrorOutOfMemory ? BLKAMG_ENOMEM : BLKAMG_EHIP,               \
                  std::string(#expr) + ": " + hipGetErrorString(e_));                     \
  } while (0)

// Wrap the body of an exported function.
#define BLK_API_BEGIN try {
#define BLK_API_END                                              \
  return BLKAMG_OK;                                              \
  }                                                              \
  catch (const ::blk::Error& e) {                                \
    ::blk::set_last_error(e.msg);                                \
    return e.code;                                               \
  }                                                              \
  catch (const std::bad_alloc&) {                                \
    ::blk::set_last_error("host allocation failed");             \
    return BLKAMG_ENOMEM;                                        \
  }                                                              \
  catch (...) {                                                  \
    ::blk::set_last_error("unexpected internal error");          \
    return BLKAMG_EINVAL;                                        \
  }

// ---------------------------------------------------------------------------
// Device allocator: hipMalloc/hipFree, or the caller's pair of routines
// ---------------------------------------------------------------------------
struct DeviceAllocator {
  blkamg_alloc_fn alloc_fn = nullptr;  // NULL: hipMalloc / hipFree
  blkamg_free_fn free_fn = nullptr;
  void* ctx = nullptr;
};
inline std::mutex& allocator_mutex() {
  static std::mutex m;
  return m;
}
inline DeviceAllocator& allocator_slot() {
  static DeviceAllocator a;
  return a;
}
inline DeviceAllocator current_allocator() {
  std::lock_guard<std::mutex> g(allocator_mutex());
  return allocator_slot();
}
constexpr uintptr_t kDevAlign = 256;

// ---------------------------------------------------------------------------
// Device buffer (owning, freed on destruction by the routine that allocated it)
// ---------------------------------------------------------------------------
template <class T>
struct DevBuf {
  T* p = nullptr;
  size_t n = 0;
  DeviceAllocator by;
  DevBuf() = default;
  explicit DevBuf(size_t count) { alloc(count); }
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : p(o.p), n(o.n), by(o.by) { o.p = nullptr; o.n = 0; }
  DevBuf& operator=(DevBuf&& o) noexcept {
    if (this != &o) { release(); p = o.p; n = o.n; by = o.by; o.p = nullptr; o.n = 0; }
    return *this;
  }
  ~DevBuf() { release(); }
  void alloc(size_t count) {
    release();
    if (count == 0) return;
    const size_t bytes = count * sizeof(T);
    const DeviceAllocator a = current_allocator();
    void* q = nullptr;
    if (a.alloc_fn) {
      q = a.alloc_fn(bytes, a.ctx);
      if (q == nullptr) fail(BLKAMG_ENOMEM, "the caller's allocator returned NULL for " + std::to_string(bytes) + " bytes");
      if (reinterpret_cast<uintptr_t>(q) % kDevAlign != 0) {
        a.free_fn(q, bytes, a.ctx);
        fail(BLKAMG_EINVAL, "the caller's allocator returned a pointer not aligned to 256 bytes");
      }
    } else {
      hipError_t e = hipMalloc(&q, bytes);
      if (e != hipSuccess) {
        (void)hipGetLastError();
        fail(BLKAMG_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
      }
    }
    p = static_cast<T*>(q);
    n = count;
    by = a;
  }
  void release() {
    if (p) {
      if (by.free_fn) {
        // as hipFree does: nothing queued may still use the buffer when it is handed back
        (void)hipDeviceSynchronize();
        by.free_fn(p, n * sizeof(T), by.ctx);
      } else {
        (void)hipFree(p);
      }
    }
    p = nullptr;
    n = 0;
  }
  size_t bytes() const { return n * sizeof(T); }
};

template <class T>
inline void upload(DevBuf<T>& d, const std::vector<T>& h) {
  d.alloc(h.size());
  if (!h.empty()) HIP_CHECK(hipMemcpy(d.p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice));
}

// Device -> host copy after all work queued on the device, whatever stream it was
// queued on (a plain hipMemcpy on the null stream does not wait for non-blocking
// streams).
template <class T>
inline std::vector<T> download(const T* d, size_t n) {
  std::vector<T> h(n);
  if (n) {
    HIP_CHECK(hipDeviceSynchronize());
    HIP_CHECK(hipMemcpy(h.data(), d, n * sizeof(T), hipMemcpyDeviceToHost));
  }
  return h;
}

// Device -> host copy ordered after the work queued on stream s.
template <class T>
inline std::vector<T> download(const T* d, size_t n, hipStream_t s) {
  std::vector<T> h(n);
  if (n) {
    HIP_CHECK(hipMemcpyAsync(h.data(), d, n * sizeof(T), hipMemcpyDeviceToHost, s));
    HIP_CHECK(hipStreamSynchronize(s));
  }
  return h;
}

inline size_t dtype_size(int dt) {
  switch (dt) {
    case BLKAMG_F64: return 8;
    case BLKAMG_F32: return 4;
    case BLKAMG_BF16: return 2;
    default: fail(BLKAMG_EINVAL, "unknown dtype " + std::to_string(dt));
  }
}

// bfloat16 stored as raw 16 bits
struct bf16 {
  uint16_t bits;
};

__host__ __device__ inline float to_float(bf16 v) {
  uint32_t u = static_cast<uint32_t>(v.bits) << 16;
  float f;
  memcpy(&f, &u, 4);
  return f;
}

// round-to-nearest-even float -> bf16 (NaN kept quiet)
__host__ __device__ inline bf16 to_bf16(float f) {
  uint32_t u;
  memcpy(&u, &f, 4);
  if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x7fffffu)) return bf16{static_cast<uint16_t>((u >> 16) | 0x40)};
  uint32_t lsb = (u >> 16) & 1u;
  u += 0x7fffu + lsb;
  return bf16{static_cast<uint16_t>(u >> 16)};
}

template <class TA>
__device__ __forceinline__ TA ld(const double* p) { return static_cast<TA>(*p); }
template <class TA>
__device__ __forceinline__ TA ld(const float* p) { return static_cast<TA>(*p); }
template <class TA>
__device__ __forceinline__ TA ld(const bf16* p) { return static_cast<TA>(to_float(*p)); }

template <class T>
__device__ __forceinline__ void st(T* p, double v) { *p = static_cast<T>(v); }
template <class T>
__device__ __forceinline__ void st(T* p, float v) { *p = static_cast<T>(v); }

// ---------------------------------------------------------------------------
// Launch geometry.  The hardware hands workgroup b to XCD (b mod 8); each XCD has
// its own L2.  Remapping so that every XCD works on one contiguous range of
// logical blocks keeps neighbouring block rows (which share gathered vector
// entries) in the same L2.
// ---------------------------------------------------------------------------
constexpr int kNumXcd = 8;

__device__ __forceinline__ int xcd_logical_block(int hw_block, int nblocks) {
  const int q = nblocks / kNumXcd, r = nblocks % kNumXcd;
  const int x = hw_block % kNumXcd, k = hw_block / kNumXcd;
  return (x < r) ? x * (q + 1) + k : r * (q + 1) + (x - r) * q + k;
}

// Rotating runs: each XCD takes runs of `chunk` consecutive logical blocks and the runs
// rotate over the XCDs.  Neighbouring blocks within a run share one L2, while all XCDs
// work near the same region at any time, so the shared MALL holds what they reuse.
// Measured on the fine 3x3 SpMV at 128^3: runs of 32-64 workgroups are 4-7 % faster
// than one contiguous range per XCD.  A bijection on 0..n-1 (the incomplete last round
// keeps the hardware order).
__device__ __forceinline__ int xcd_chunked_block(int hw_block, int nblocks, int chunk) {
  const int round = kNumXcd * chunk;
  const int full = (nblocks / round) * round;
  if (hw_block >= full) return hw_block;
  const int x = hw_block % kNumXcd, k = hw_block / kNumXcd;
  return (k / chunk) * round + x * chunk + (k % chunk);
}
constexpr int kSpmvChunk = 64;

inline int ceil_div(int64_t a, int64_t b) { return static_cast<int>((a + b - 1) / b); }

// sum over the G lanes of a group (G a power of two <= 64), result in all lanes
template <int G, class T>
__device__ __forceinline__ T group_sum(T v) {
#pragma unroll
  for (int off = G / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, G);
  return v;
}

// Deterministic sum over a 256-thread block; every thread contributes v, thread 0
// gets the result (fixed order: wave tree, then the 4 waves in order).
__device__ __forceinline__ double block_sum_256(double v, double* lds4) {
  v = group_sum<64>(v);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) lds4[w] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) s = ((lds4[0] + lds4[1]) + lds4[2]) + lds4[3];
  return s;
}

hipStream_t as_stream(void* s);

}  // namespace blk

// Common helpers for the gfx950 projection solver: error reporting, device
// buffers and deterministic reductions (no floating-point atomics anywhere, so
// every coefficient is reproducible run to run and the second Lanczos pass can
// replay the first one exactly).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "lyap.h"

namespace lyap {

// ------------------------------------------------------------------ errors
void set_error(const char* fmt, ...);
void clear_error();

struct Error {
  lyap_status st;
};

#define LYAP_HIP(expr)                                                              \
  do {                                                                              \
    hipError_t e_ = (expr);                                                         \
    if (e_ != hipSuccess) {                                                         \
      ::lyap::set_error("%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_),     \
                        __FILE__, __LINE__);                                        \
      throw ::lyap::Error{e_ == hipErrorOutOfMemory ? LYAP_E_NOMEM : LYAP_E_DEVICE}; \
    }                                                                               \
  } while (0)

#define LYAP_REQUIRE(cond, status, ...) \
  do {                                  \
    if (!(cond)) {                      \
      ::lyap::set_error(__VA_ARGS__);   \
      throw ::lyap::Error{status};      \
    }                                   \
  } while (0)

// Launch check: a failed launch reports the kernel name.
#define LYAP_LAUNCHED(name) LYAP_HIP(hipGetLastError())

// ------------------------------------------------------------------ buffers
// Owning device buffer (hipMalloc / hipFree).  Sizes in bytes.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  explicit DevBuf(size_t b) { alloc(b); }
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : p(o.p), bytes(o.bytes) { o.p = nullptr; o.bytes = 0; }
  DevBuf& operator=(DevBuf&& o) noexcept {
    if (this != &o) { release(); p = o.p; bytes = o.bytes; o.p = nullptr; o.bytes = 0; }
    return *this;
  }
  ~DevBuf() { release(); }
  void alloc(size_t b) {
    release();
    if (b == 0) b = 256;
    hipError_t e = hipMalloc(&p, b);
    if (e != hipSuccess) {
      p = nullptr;
      set_error("hipMalloc(%zu bytes) failed: %s", b, hipGetErrorString(e));
      throw Error{LYAP_E_NOMEM};
    }
    bytes = b;
  }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  template <typename U> U* as() const { return static_cast<U*>(p); }
};

// Pinned host buffer (hipHostMalloc).
struct HostBuf {
  void* p = nullptr;
  size_t bytes = 0;
  HostBuf() = default;
  explicit HostBuf(size_t b) {
    LYAP_HIP(hipHostMalloc(&p, b ? b : 64, hipHostMallocDefault));
    bytes = b;
  }
  HostBuf(const HostBuf&) = delete;
  HostBuf& operator=(const HostBuf&) = delete;
  ~HostBuf() { if (p) (void)hipHostFree(p); }
  template <typename U> U* as() const { return static_cast<U*>(p); }
};

// ------------------------------------------------------------------ reductions
constexpr int kBlock = 256;          // threads per workgroup of the streaming kernels
constexpr int kWaves = kBlock / 64;  // wave64

// Sum of v over the 64 lanes of a wave (butterfly, fixed order).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Reduce K per-thread values over a kBlock-thread workgroup.  The result is in
// red[0..K) (shared memory, K*kWaves doubles of scratch); deterministic.
template <int K>
__device__ __forceinline__ void block_sum(double (&v)[K], double* red /* K*kWaves */) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    double s = wave_sum(v[k]);
    if (lane == 0) red[wave * K + k] = s;
  }
  __syncthreads();
  if (threadIdx.x < K) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) s += red[w * K + threadIdx.x];
    red[threadIdx.x] = s;  // rows w>0 are not read again; row 0 slot k is only
                           // rewritten by thread k after it read it.
  }
  __syncthreads();
}

// Grid-wide reduction epilogue ("last workgroup finishes"): every workgroup
// writes its K partial sums to part[blockIdx.x*K..], then the workgroup that
// arrives last sums all partials in a fixed order and returns true with the
// totals in red[0..K).  The arrival counter is reset for the next launch.
template <int K>
__device__ __forceinline__ bool grid_sum_last(double (&v)[K], double* red, double* part,
                                              unsigned* counter) {
  block_sum<K>(v, red);
  __shared__ bool last;
  if (threadIdx.x < K) part[(size_t)blockIdx.x * K + threadIdx.x] = red[threadIdx.x];
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned prev = atomicAdd(counter, 1u);
    last = (prev == gridDim.x - 1);
  }
  __syncthreads();
  if (!last) return false;
  __threadfence();
  double acc[K];
#pragma unroll
  for (int k = 0; k < K; ++k) acc[k] = 0.0;
  for (unsigned b = threadIdx.x; b < gridDim.x; b += kBlock) {
#pragma unroll
    for (int k = 0; k < K; ++k) acc[k] += __builtin_nontemporal_load(&part[(size_t)b * K + k]);
  }
  __syncthreads();
  block_sum<K>(acc, red);
  if (threadIdx.x == 0) *counter = 0u;
  return true;
}

inline int grid_for(int64_t rows, int rows_per_thread_min = 1, int max_blocks = 2048) {
  int64_t b = (rows + (int64_t)kBlock * rows_per_thread_min - 1) / ((int64_t)kBlock * rows_per_thread_min);
  if (b < 1) b = 1;
  if (b > max_blocks) b = max_blocks;
  return (int)b;
}

}  // namespace lyap

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
constexpr int kBlock = 256;          // threads per workgroup of the small kernels
constexpr int kWaves = kBlock / 64;  // wave64

// Sum of v over the 64 lanes of a wave (butterfly, fixed order; every lane
// ends with the total).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

constexpr int pow2_at_least(int k) {
  int p = 1;
  while (p < k) p <<= 1;
  return p;
}

// Sums of K per-lane values over a wave with a "transpose" butterfly: at each
// step a lane keeps half of its values and receives the partner's copy of
// that half, so K values need K-1 (+ the remaining log steps) shuffles instead
// of K*6.  Returns the wave total of value index key(lane) in every lane; the
// lanes whose low bits (below 64/P) are zero hold distinct keys 0..P-1.
template <int K>
__device__ __forceinline__ double wave_transpose_sum(const double (&v)[K], int lane, int* key) {
  constexpr int P = pow2_at_least(K);
  double w[P];
#pragma unroll
  for (int i = 0; i < P; ++i) w[i] = i < K ? v[i] : 0.0;
  int k = 0;
  int off = 32;
#pragma unroll
  for (int cnt = P; cnt > 1; cnt >>= 1) {
    const int half = cnt >> 1;
    const bool up = (lane & off) != 0;
#pragma unroll
    for (int i = 0; i < half; ++i) {
      const double send = up ? w[i] : w[i + half];
      const double keep = up ? w[i + half] : w[i];
      w[i] = keep + __shfl_xor(send, off, 64);
    }
    if (up) k += half;
    off >>= 1;
  }
  double r = w[0];
  for (; off > 0; off >>= 1) r += __shfl_xor(r, off, 64);
  *key = k;
  return r;
}

// Reduce K per-thread values over an NT-thread workgroup.  The result is in
// red[0..K) (shared memory, pow2(K)*(NT/64) doubles of scratch); deterministic.
template <int K, int NT = kBlock>
__device__ __forceinline__ void block_sum(double (&v)[K], double* red) {
  constexpr int W = NT / 64;
  constexpr int P = pow2_at_least(K);
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  int key;
  const double s = wave_transpose_sum<K>(v, lane, &key);
  if ((lane & ((64 / P) - 1)) == 0 && key < K) red[wave * P + key] = s;
  __syncthreads();
  if (threadIdx.x < K) {
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < W; ++w) t += red[w * P + threadIdx.x];
    red[threadIdx.x] = t;  // slot k is only rewritten by thread k after reading it
  }
  __syncthreads();
}

// Grid-wide reduction epilogue ("last workgroup finishes", used by the small
// check kernels): every workgroup writes its K partial sums, the last one to
// arrive sums them in a fixed order and returns true with the totals in
// red[0..K).  The arrival counter is reset for the next launch.
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

// A value known to be identical in every lane, moved to a scalar register.
__device__ __forceinline__ double uniform_d(double v) {
  const long long x = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readfirstlane((int)(x & 0xffffffffll));
  const int hi = __builtin_amdgcn_readfirstlane((int)(x >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Streaming kernels of the Lanczos step: one 1024-thread workgroup per CU.
// Each writes one partial Gram matrix per workgroup with plain stores; the
// next kernel in the stream reduces all partials in its prologue (every
// workgroup in the same fixed order, so all see bit-identical totals).  Kernel
// boundaries order the accesses, so no atomics or device-scope fences are
// needed.
constexpr int kSBlock = 1024;
constexpr int kSGrid = 256;
// Block widths above 4 keep S*S FP64 accumulators and coefficients per thread:
// those kernels run 256-thread workgroups (one wave per SIMD, full register file).
constexpr int stream_threads(int S) { return S <= 4 ? kSBlock : 256; }

template <int K, int NT>
__device__ __forceinline__ void reduce_partials(const double* __restrict__ part, int nparts, double* red) {
  // thread -> (value k, group of partials); the groups of one k are then summed
  // across lanes and waves, always in the same order
  constexpr int P = pow2_at_least(K);
  static_assert(P <= 64, "K too large");
  constexpr int G = NT / P;  // partial groups
  const int k = threadIdx.x & (P - 1);
  const int grp = threadIdx.x / P;
  double acc = 0.0;
  if (k < K)
    for (int b = grp; b < nparts; b += G) acc += part[(size_t)b * K + k];
  // lanes with the same k within a wave: offsets P..32
  for (int off = 32; off >= P; off >>= 1) acc += __shfl_xor(acc, off, 64);
  constexpr int W = NT / 64;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane < P && k < K) red[wave * P + k] = acc;
  __syncthreads();
  if (threadIdx.x < K) {
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < W; ++w) t += red[w * P + threadIdx.x];
    red[threadIdx.x] = t;
  }
  __syncthreads();
}

template <int K, int NT>
__device__ __forceinline__ void write_partial(double (&v)[K], double* red, double* part) {
  block_sum<K, NT>(v, red);
  if (threadIdx.x < K) part[(size_t)blockIdx.x * K + threadIdx.x] = red[threadIdx.x];
}

inline int grid_for(int64_t rows, int rows_per_thread_min = 1, int max_blocks = 2048) {
  int64_t b = (rows + (int64_t)kBlock * rows_per_thread_min - 1) / ((int64_t)kBlock * rows_per_thread_min);
  if (b < 1) b = 1;
  if (b > max_blocks) b = max_blocks;
  return (int)b;
}

}  // namespace lyap

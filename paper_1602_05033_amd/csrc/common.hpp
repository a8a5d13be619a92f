// Common helpers for the gfx950 projection solver: error reporting, device
// buffers and deterministic reductions (no floating-point atomics anywhere, so
// every coefficient is reproducible run to run and the second Lanczos pass can
// replay the first one exactly).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <cstring>
#include <exception>
#include <map>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "lyap.h"

namespace lyap {

// ------------------------------------------------------------------ errors
void set_error(const char* fmt, ...);
void clear_error();
const char* last_error();

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
// Caller-provided device workspace.  While an Arena is installed on the
// calling thread (ArenaScope), every DevBuf takes its bytes from it by bump
// allocation (256-byte aligned) instead of hipMalloc, and gives nothing back
// on release; a request past the capacity throws LYAP_E_ARG.
struct Arena {
  char* base = nullptr;
  size_t cap = 0;
  size_t used = 0;
};

inline Arena*& current_arena() {
  static thread_local Arena* a = nullptr;
  return a;
}

struct ArenaScope {
  explicit ArenaScope(Arena* a) : prev_(current_arena()) { current_arena() = a; }
  ~ArenaScope() { current_arena() = prev_; }
  ArenaScope(const ArenaScope&) = delete;
  ArenaScope& operator=(const ArenaScope&) = delete;

 private:
  Arena* prev_;
};

// Device block cache.  While a BlockCacheScope is installed on the calling
// thread, DevBuf takes its memory from a process-wide cache of released blocks
// (per device, sizes rounded up to a quarter of their power of two) and gives
// it back there instead of calling hipMalloc / hipFree, which are slow and
// make the device wait.  Code that installs the scope must release a buffer
// only once no kernel can still use it (the guarantee hipFree's wait would
// otherwise give); during exception unwinding blocks are freed for real.
class BlockCache {
 public:
  static BlockCache& get() {
    static BlockCache c;
    return c;
  }
  static size_t size_class(size_t b) {
    size_t c = 4096;
    while (c < b) c <<= 1;
    if (c > 16384) {  // quarters of the power of two
      const size_t q = c / 8;
      size_t r = c / 2;
      while (r < b) r += q;
      c = r;
    }
    return c;
  }
  void* take(int dev, size_t cls) {
    std::lock_guard<std::mutex> g(mu_);
    auto it = free_.find(std::make_pair(dev, cls));
    if (it == free_.end()) return nullptr;
    void* p = it->second;
    free_.erase(it);
    held_ -= cls;
    return p;
  }
  // false: the cache is full, the caller frees the block
  bool give(int dev, size_t cls, void* p) {
    std::lock_guard<std::mutex> g(mu_);
    if (held_ + cls > kMaxHeld) return false;
    free_.emplace(std::make_pair(dev, cls), p);
    held_ += cls;
    return true;
  }

 private:
  static constexpr size_t kMaxHeld = size_t(8) << 30;  // bytes kept for reuse
  std::mutex mu_;
  std::multimap<std::pair<int, size_t>, void*> free_;
  size_t held_ = 0;
};

inline bool& block_cache_on() {
  static thread_local bool on = false;
  return on;
}

struct BlockCacheScope {
  BlockCacheScope() : prev_(block_cache_on()) { block_cache_on() = true; }
  ~BlockCacheScope() { block_cache_on() = prev_; }
  BlockCacheScope(const BlockCacheScope&) = delete;
  BlockCacheScope& operator=(const BlockCacheScope&) = delete;

 private:
  bool prev_;
};

// Owning device buffer (hipMalloc / hipFree, a block of the BlockCache, or a
// slice of the installed Arena).  Sizes in bytes.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  bool borrowed = false;  // slice of an Arena: never freed
  size_t cached = 0;      // size class of a BlockCache block (0: own allocation)
  int dev = 0;
  DevBuf() = default;
  explicit DevBuf(size_t b) { alloc(b); }
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : p(o.p), bytes(o.bytes), borrowed(o.borrowed), cached(o.cached), dev(o.dev) {
    o.p = nullptr;
    o.bytes = 0;
    o.borrowed = false;
    o.cached = 0;
  }
  DevBuf& operator=(DevBuf&& o) noexcept {
    if (this != &o) {
      release();
      p = o.p;
      bytes = o.bytes;
      borrowed = o.borrowed;
      cached = o.cached;
      dev = o.dev;
      o.p = nullptr;
      o.bytes = 0;
      o.borrowed = false;
      o.cached = 0;
    }
    return *this;
  }
  ~DevBuf() { release(); }
  void alloc(size_t b) {
    release();
    if (b == 0) b = 256;
    if (Arena* a = current_arena()) {
      const size_t off = (a->used + 255) / 256 * 256;
      if (off > a->cap || b > a->cap - off) {
        set_error("workspace exhausted: %zu more bytes needed beyond %zu of %zu", b, off, a->cap);
        throw Error{LYAP_E_ARG};
      }
      p = a->base + off;
      a->used = off + b;
      bytes = b;
      borrowed = true;
      return;
    }
    size_t req = b;
    if (block_cache_on()) {
      (void)hipGetDevice(&dev);
      req = BlockCache::size_class(b);
      p = BlockCache::get().take(dev, req);
      if (p) {
        bytes = b;
        cached = req;
        return;
      }
    }
    hipError_t e = hipMalloc(&p, req);
    if (e != hipSuccess) {
      p = nullptr;
      set_error("hipMalloc(%zu bytes) failed: %s", req, hipGetErrorString(e));
      throw Error{LYAP_E_NOMEM};
    }
    bytes = b;
    cached = block_cache_on() ? req : 0;
  }
  void release() {
    if (p && !borrowed) {
      // a cached block goes back to the cache, except while an exception
      // unwinds (work may still be in flight: hipFree waits for it)
      if (!(cached && std::uncaught_exceptions() == 0 && BlockCache::get().give(dev, cached, p))) (void)hipFree(p);
    }
    p = nullptr;
    bytes = 0;
    borrowed = false;
    cached = 0;
  }
  template <typename U> U* as() const { return static_cast<U*>(p); }
};

// Pinned host buffer (hipHostMalloc).
struct HostBuf {
  void* p = nullptr;
  size_t bytes = 0;
  HostBuf() = default;
  explicit HostBuf(size_t b) { alloc(b); }
  void alloc(size_t b) {
    if (p) (void)hipHostFree(p);
    p = nullptr;
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

// ------------------------------------------------------------------ cross-lane exchange
// Value held by lane (l ^ M) of the same wave, without going through the LDS
// crossbar (ds_bpermute costs tens of cycles of LDS time per instruction and
// dominated every reduction epilogue): DPP row permutations inside each
// 16-lane row -- quad_perm [1,0,3,2] (M = 1), [2,3,0,1] (M = 2), the half-row
// mirror (lane i <-> 7 - i, M = 7) and the row mirror (i <-> 15 - i, M = 15)
// -- and the gfx950 permlane swaps across rows (M = 16, 32), which return the
// even-row / low-half copy first.  All are plain VALU instructions.
template <int M>
__device__ __forceinline__ unsigned lane_xor_u(unsigned x) {
  static_assert(M == 1 || M == 2 || M == 7 || M == 15 || M == 16 || M == 32, "unsupported lane mask");
  if constexpr (M == 1) {
    return (unsigned)__builtin_amdgcn_update_dpp(0, (int)x, 0xB1, 0xF, 0xF, false);
  } else if constexpr (M == 2) {
    return (unsigned)__builtin_amdgcn_update_dpp(0, (int)x, 0x4E, 0xF, 0xF, false);
  } else if constexpr (M == 7) {
    return (unsigned)__builtin_amdgcn_update_dpp(0, (int)x, 0x141, 0xF, 0xF, false);
  } else if constexpr (M == 15) {
    return (unsigned)__builtin_amdgcn_update_dpp(0, (int)x, 0x140, 0xF, 0xF, false);
  } else if constexpr (M == 16) {
    const auto s = __builtin_amdgcn_permlane16_swap(x, x, false, false);  // {even rows, odd rows}
    return (__lane_id() & 16) ? s[0] : s[1];
  } else {
    const auto s = __builtin_amdgcn_permlane32_swap(x, x, false, false);  // {low half, high half}
    return (__lane_id() & 32) ? s[0] : s[1];
  }
}

template <int M>
__device__ __forceinline__ double lane_xor(double v) {
  const unsigned long long x = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = lane_xor_u<M>((unsigned)(x & 0xffffffffull));
  const unsigned hi = lane_xor_u<M>((unsigned)(x >> 32));
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

template <int M>
__device__ __forceinline__ int lane_xor(int v) {
  return (int)lane_xor_u<M>((unsigned)v);
}

// Butterfly over the 64 lanes (masks 1, 2, 7, 15, 16, 32 span all six lane
// bits).  Each lane combines its value with its partner's; the combination is
// commutative, so both lanes of a pair hold the same bits and every lane ends
// with the identical total.
__device__ __forceinline__ double wave_sum(double v) {
  v += lane_xor<1>(v);
  v += lane_xor<2>(v);
  v += lane_xor<7>(v);
  v += lane_xor<15>(v);
  v += lane_xor<16>(v);
  v += lane_xor<32>(v);
  return v;
}

// Sum over aligned groups of G lanes (G a power of two <= 64): the first
// log2(G) butterfly steps of wave_sum; every lane gets its group's sum.
template <int G>
__device__ __forceinline__ double group_sum(double v) {
  if constexpr (G >= 2) v += lane_xor<1>(v);
  if constexpr (G >= 4) v += lane_xor<2>(v);
  if constexpr (G >= 8) v += lane_xor<7>(v);
  if constexpr (G >= 16) v += lane_xor<15>(v);
  if constexpr (G >= 32) v += lane_xor<16>(v);
  if constexpr (G >= 64) v += lane_xor<32>(v);
  return v;
}

__device__ __forceinline__ double wave_max(double v) {
  v = fmax(v, lane_xor<1>(v));
  v = fmax(v, lane_xor<2>(v));
  v = fmax(v, lane_xor<7>(v));
  v = fmax(v, lane_xor<15>(v));
  v = fmax(v, lane_xor<16>(v));
  v = fmax(v, lane_xor<32>(v));
  return v;
}

__device__ __forceinline__ double wave_prod(double v) {
  v *= lane_xor<1>(v);
  v *= lane_xor<2>(v);
  v *= lane_xor<7>(v);
  v *= lane_xor<15>(v);
  v *= lane_xor<16>(v);
  v *= lane_xor<32>(v);
  return v;
}

constexpr int pow2_at_least(int k) {
  int p = 1;
  while (p < k) p <<= 1;
  return p;
}

constexpr int log2_exact(int p) {
  int l = 0;
  while ((1 << l) < p) ++l;
  return l;
}

// One step of the transpose butterfly on lane bit B (partner mask M flips B
// and only lower bits): the lane keeps the half of its CNT values selected by
// bit B, adds the partner's copy of that half, and records the key offset.
template <int M, int B, int CNT>
__device__ __forceinline__ void transpose_step(double* w, int lane, int& key) {
  constexpr int H = CNT / 2;
  const bool up = ((lane >> B) & 1) != 0;
#pragma unroll
  for (int i = 0; i < H; ++i) {
    const double send = up ? w[i] : w[i + H];
    const double keep = up ? w[i + H] : w[i];
    w[i] = keep + lane_xor<M>(send);
  }
  if (up) key += H;
}

// Sum of v over the 64 lanes of a wave for P = pow2(K) values per lane.  Within
// each 16-lane row a transpose butterfly on lane bits 3, 2, 1, 0 halves the
// values held per lane at each step (P - 1 exchanges for P values instead of
// 6 P); the remaining bits are plain sums, then the four rows are combined.
// On return lane l holds the wave totals of keys key .. key + C - 1 in w[0..C),
// C = max(P / 16, 1); in row 0 the lanes with (l & (16 / P - 1)) == 0 hold
// each key exactly once.
template <int P>
__device__ __forceinline__ void wave_transpose_sum(double* w, int lane, int& key) {
  key = 0;
  if constexpr (P >= 2) transpose_step<15, 3, P>(w, lane, key);
  else w[0] += lane_xor<15>(w[0]);
  if constexpr (P >= 4) transpose_step<7, 2, P / 2>(w, lane, key);
  else w[0] += lane_xor<7>(w[0]);
  if constexpr (P >= 8) transpose_step<2, 1, P / 4>(w, lane, key);
  else w[0] += lane_xor<2>(w[0]);
  if constexpr (P >= 16) transpose_step<1, 0, P / 8>(w, lane, key);
  else w[0] += lane_xor<1>(w[0]);
  constexpr int C = P >= 16 ? P / 16 : 1;
#pragma unroll
  for (int i = 0; i < C; ++i) {
    w[i] += lane_xor<16>(w[i]);
    w[i] += lane_xor<32>(w[i]);
  }
}

// Reduce K per-thread values over an NT-thread workgroup.  The result is in
// red[0..K) (shared memory, pow2(K)*(NT/64) doubles of scratch); deterministic.
template <int K, int NT = kBlock>
__device__ __forceinline__ void block_sum(double (&v)[K], double* red) {
  constexpr int W = NT / 64;
  constexpr int P = pow2_at_least(K);
  constexpr int C = P >= 16 ? P / 16 : 1;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  double w[P];
#pragma unroll
  for (int i = 0; i < P; ++i) w[i] = i < K ? v[i] : 0.0;
  int key;
  wave_transpose_sum<P>(w, lane, key);
  constexpr int lowmask = P >= 16 ? 0 : 16 / P - 1;
  if (lane < 16 && (lane & lowmask) == 0) {
#pragma unroll
    for (int i = 0; i < C; ++i)
      if (key + i < K) red[wave * P + key + i] = w[i];
  }
  __syncthreads();
  if (threadIdx.x < K) {
    double t = 0.0;
#pragma unroll
    for (int q = 0; q < W; ++q) t += red[q * P + threadIdx.x];
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
  // lane -> (value k in the high lane bits, slot in the low bits); the slots of
  // one k are summed over the low lane bits and then across waves, always in
  // the same order
  constexpr int P = pow2_at_least(K);
  static_assert(P <= 64, "K too large");
  constexpr int LB = 6 - log2_exact(P);  // low lane bits = slots per wave
  constexpr int G = NT / P;              // slots in the workgroup
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int k = lane >> LB;
  const int g = wave * (1 << LB) + (lane & ((1 << LB) - 1));
  double acc = 0.0;
  if (k < K)
    for (int b = g; b < nparts; b += G) acc += part[(size_t)b * K + k];
  if constexpr (LB >= 1) acc += lane_xor<1>(acc);
  if constexpr (LB >= 2) acc += lane_xor<2>(acc);
  if constexpr (LB >= 3) acc += lane_xor<7>(acc);
  if constexpr (LB >= 4) acc += lane_xor<15>(acc);
  if constexpr (LB >= 5) acc += lane_xor<16>(acc);
  if constexpr (LB >= 6) acc += lane_xor<32>(acc);
  constexpr int W = NT / 64;
  if ((lane & ((1 << LB) - 1)) == 0 && k < K) red[wave * P + k] = acc;
  __syncthreads();
  if (threadIdx.x < K) {
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < W; ++w) t += red[w * P + threadIdx.x];
    red[threadIdx.x] = t;
  }
  __syncthreads();
}

// Two scalar totals at once: red[0] = sum of a[0..na), red[1] = sum of
// b[0..nb), each added in exactly the order of reduce_partials<1, NT> (the
// same bits), with the loads of both arrays in flight together and one pair of
// barriers instead of two.
template <int NT>
__device__ __forceinline__ void reduce_partials_pair(const double* __restrict__ a, int na,
                                                     const double* __restrict__ b, int nb, double* red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = threadIdx.x;
  double sa = 0.0, sb = 0.0;
  for (int i = g; i < na; i += NT) sa += a[i];
  for (int i = g; i < nb; i += NT) sb += b[i];
  sa += lane_xor<1>(sa);
  sb += lane_xor<1>(sb);
  sa += lane_xor<2>(sa);
  sb += lane_xor<2>(sb);
  sa += lane_xor<7>(sa);
  sb += lane_xor<7>(sb);
  sa += lane_xor<15>(sa);
  sb += lane_xor<15>(sb);
  sa += lane_xor<16>(sa);
  sb += lane_xor<16>(sb);
  sa += lane_xor<32>(sa);
  sb += lane_xor<32>(sb);
  constexpr int W = NT / 64;
  if (lane == 0) {
    red[wave] = sa;
    red[W + wave] = sb;
  }
  __syncthreads();
  if (threadIdx.x < 2) {
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < W; ++w) t += red[threadIdx.x * W + w];
    red[2 * W + threadIdx.x] = t;
  }
  __syncthreads();
  if (threadIdx.x < 2) red[threadIdx.x] = red[2 * W + threadIdx.x];
  __syncthreads();
}

template <int K, int NT>
__device__ __forceinline__ void write_partial_at(double (&v)[K], double* red, double* part, int idx) {
  block_sum<K, NT>(v, red);
  if (threadIdx.x < K) part[(size_t)idx * K + threadIdx.x] = red[threadIdx.x];
}

template <int K, int NT>
__device__ __forceinline__ void write_partial(double (&v)[K], double* red, double* part) {
  write_partial_at<K, NT>(v, red, part, blockIdx.x);
}

inline int grid_for(int64_t rows, int rows_per_thread_min = 1, int max_blocks = 2048) {
  int64_t b = (rows + (int64_t)kBlock * rows_per_thread_min - 1) / ((int64_t)kBlock * rows_per_thread_min);
  if (b < 1) b = 1;
  if (b > max_blocks) b = max_blocks;
  return (int)b;
}

}  // namespace lyap

// Block Lanczos on gfx950: one step of Algorithm 2 as a chain of streaming
// kernels over row-interleaved n x S blocks, each fusing the update of W with
// the next Gram product so that W is read and written once per MGS stage:
//
//   K1  W  = A V_j                         ; alpha1 = V_{j-1}^T W
//   K2  W -= V_{j-1} alpha1                ; alpha2 = V_j^T W
//   K3  W -= V_j alpha2                    ; alpha3 = V_{j-1}^T W
//   K4  W -= V_{j-1} alpha3                ; alpha4 = V_j^T W
//   K5  W -= V_j alpha4                    ; G1 = W^T W -> R1 (Cholesky)
//   K6  U  = W R1^{-1} (not stored)        ; G2 = U^T U -> R2, tau_{j+1,j} = R2 R1
//   K7  V_{j+1} = W (R1^{-1} R2^{-1})
//
// i.e. block MGS applied twice against V_{j-1} then V_j (Algorithm 2 steps
// 2-8) followed by the economy QR of step 9 done as Cholesky-QR twice (the
// positive-diagonal QR factor).  Gram products accumulate in FP64 whatever the
// storage type; every update is evaluated in FP64 and rounded once to the
// storage type.  Each kernel's last workgroup reduces the partial Gram
// matrices in a fixed order and writes the coefficient to the step log, so the
// log is bit-reproducible; the second pass (replay) reapplies exactly the
// same per-row arithmetic with the logged coefficients (Section 3.3) and
// regenerates every block bit for bit.
#include "lanczos.hpp"
#include "small.hpp"

namespace lyap {

// ------------------------------------------------------------------ per-row arithmetic
template <typename T, int S>
__device__ __forceinline__ void upd_row(T (&w)[S], const T (&x)[S], const double* __restrict__ al) {
#pragma unroll
  for (int b = 0; b < S; ++b) {
    double acc = (double)w[b];
#pragma unroll
    for (int a = 0; a < S; ++a) acc = fma(-(double)x[a], al[a * S + b], acc);
    w[b] = (T)acc;
  }
}

template <typename T, int S>
__device__ __forceinline__ void apply_upper_d(const T (&w)[S], const double* __restrict__ Ri, double (&u)[S]) {
#pragma unroll
  for (int b = 0; b < S; ++b) {
    double acc = 0.0;
#pragma unroll
    for (int a = 0; a <= b; ++a) acc = fma((double)w[a], Ri[a * S + b], acc);
    u[b] = acc;
  }
}

template <typename T, int S>
__device__ __forceinline__ void apply_upper(const T (&w)[S], const double* __restrict__ Ri, T (&v)[S]) {
  double u[S];
  apply_upper_d<T, S>(w, Ri, u);
#pragma unroll
  for (int b = 0; b < S; ++b) v[b] = (T)u[b];
}

template <int S>
__device__ __forceinline__ void load_coef(const double* __restrict__ src, double (&dst)[S * S]) {
  // the coefficients are the same for every lane: read them through the
  // constant address space from a wave-uniform address, so that they become
  // scalar loads (SGPR operands) also when the pointer was itself loaded from
  // memory (the grouped kernels' descriptors), where it would otherwise be a
  // generic pointer and the loads per-lane
  const unsigned long long a = reinterpret_cast<unsigned long long>(src);
  const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)(a & 0xffffffffull));
  const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(a >> 32));
  using cptr = const __attribute__((address_space(4))) double*;
  const cptr c = (cptr)(((unsigned long long)hi << 32) | lo);
#pragma unroll
  for (int i = 0; i < S * S; ++i) dst[i] = c[i];
}

// ------------------------------------------------------------------ kernels
// Rows owned by this thread: grid-stride over kSBlock-thread workgroups,
// kRPT rows at a time (loads of all kRPT rows are issued before any arithmetic).
#define LYAP_ROWS(r, n) for (int r = blockIdx.x * stream_threads(S) + threadIdx.x; r < (n); r += gridDim.x * stream_threads(S))
// rows per thread: at most 64 bytes of each streamed array in flight per thread
// (measured on MI355X: one row per thread per grid-stride iteration streams at
// the cache/HBM rate; batching several rows per thread before any use was
// several times slower)
template <typename T, int S>
constexpr int rows_per_thread() {
  return 1;
}
// (wg_id, wg_cnt): this workgroup's index among the wg_cnt that share the
// problem -- blockIdx.x / gridDim.x for a single problem, the work-map entry
// in a grouped launch over several problems.
#define LYAP_BATCH(r0, n) \
  constexpr int kRPT = rows_per_thread<T, S>(); \
  for (int r0 = wg_id * NT + threadIdx.x; r0 < (n); r0 += wg_cnt * NT * kRPT)
#define LYAP_FOR_U _Pragma("unroll") for (int u = 0; u < kRPT; ++u)

template <int S>
__device__ __forceinline__ void zero(double (&a)[S * S]) {
#pragma unroll
  for (int i = 0; i < S * S; ++i) a[i] = 0.0;
}

template <typename X, typename Y, int S>
__device__ __forceinline__ void outer_acc(double (&acc)[S * S], const X (&x)[S], const Y (&y)[S]) {
#pragma unroll
  for (int p = 0; p < S; ++p)
#pragma unroll
    for (int q = 0; q < S; ++q) acc[p * S + q] = fma((double)x[p], (double)y[q], acc[p * S + q]);
}

// Prologue: total of the previous kernel's partial Gram matrices into g[];
// workgroup 0 also records it in the log slot (if slot >= 0).
template <int S, int NT = stream_threads(S)>
__device__ __forceinline__ void take_gram(const double* pin, int nparts, double* red, double (&g)[S * S],
                                          double* log_slot, bool lead) {
  reduce_partials<S * S, NT>(pin, nparts, red);
#pragma unroll
  for (int i = 0; i < S * S; ++i) g[i] = uniform_d(red[i]);
  if (lead && log_slot && threadIdx.x < S * S) log_slot[threadIdx.x] = red[threadIdx.x];
  __syncthreads();  // red is reused by the epilogue
}

// K1: W = A V_j ; partial alpha1 = V_{j-1}^T W
template <typename T, int S, int NT = stream_threads(S)>
__device__ __forceinline__ void spmm_gram_body(const StepArgs<T>& a, int wg_id, int wg_cnt, double* red) {
  double acc[S * S];
  zero<S>(acc);
  int lo, hi;
  op_rows(wg_id, wg_cnt, a.n, lo, hi);
  for (int r = lo + threadIdx.x; r < hi; r += NT) {
    T w[S], x[S];
    op_row<T, S>(a.op, a.Vcur, r, w);
    load_row<T, S>(a.Vprev + (size_t)r * S, x);
    store_row<T, S>(a.W + (size_t)r * S, w);
    outer_acc<T, T, S>(acc, x, w);
  }
  write_partial_at<S * S, NT>(acc, red, a.pout, wg_id);
}

// K2..K5: alpha_in = total of the previous partials (logged), W -= X alpha_in,
// partial Y^T W (Y == nullptr: W^T W for the QR that follows).
template <typename T, int S, int NT = stream_threads(S)>
__device__ __forceinline__ void upd_gram_body(const StepArgs<T>& a, const T* X, const T* Y, int slot_in, int wg_id,
                                              int wg_cnt, double* red) {
  double al[S * S];
  take_gram<S, NT>(a.pin, a.nparts, red, al, a.log + slot_in * S * S, wg_id == 0);
  double acc[S * S];
  zero<S>(acc);
  const int str = wg_cnt * NT;
  LYAP_BATCH(r0, a.n) {
    T w[kRPT][S], x[kRPT][S], y[kRPT][S];
    LYAP_FOR_U {
      const int r = r0 + u * str;
      if (r < a.n) {
        load_row<T, S>(a.W + (size_t)r * S, w[u]);
        load_row<T, S>(X + (size_t)r * S, x[u]);
        if (Y) load_row<T, S>(Y + (size_t)r * S, y[u]);
      }
    }
    LYAP_FOR_U {
      const int r = r0 + u * str;
      if (r < a.n) {
        upd_row<T, S>(w[u], x[u], al);
        store_row<T, S>(a.W + (size_t)r * S, w[u]);
        if (Y) outer_acc<T, T, S>(acc, y[u], w[u]);
        else outer_acc<T, T, S>(acc, w[u], w[u]);
      }
    }
  }
  write_partial_at<S * S, NT>(acc, red, a.pout, wg_id);
}

// Block classical Gram-Schmidt, twice (blocks of at most 4 columns): each
// sweep takes both coefficient blocks [V_{j-1}, V_j]^T W from one Gram pass
// and applies them in one update pass, in the order the replay uses
// (W -= V_{j-1} a1, then W -= V_j a2).  a1, a2 equal the block modified
// Gram-Schmidt coefficients up to rounding (V_j^T V_{j-1} is O(u)).
constexpr bool cgs2_width(int S) { return S <= 4; }

// Prologue of a CGS2 sweep: both coefficient blocks from the previous
// kernel's 2 S x S partials, logged in slot1 / slot2 by workgroup 0.
template <int S, int NT = stream_threads(S)>
__device__ __forceinline__ void take_gram2(const double* pin, int nparts, double* red, double (&g1)[S * S],
                                           double (&g2)[S * S], double* log1, double* log2, bool lead) {
  reduce_partials<2 * S * S, NT>(pin, nparts, red);
#pragma unroll
  for (int i = 0; i < S * S; ++i) {
    g1[i] = uniform_d(red[i]);
    g2[i] = uniform_d(red[S * S + i]);
  }
  if (lead && threadIdx.x < S * S) {
    log1[threadIdx.x] = red[threadIdx.x];
    log2[threadIdx.x] = red[S * S + threadIdx.x];
  }
  __syncthreads();  // red is reused by the epilogue
}

// K1 (CGS2): W = A V_j ; partials [V_{j-1}, V_j]^T W
template <typename T, int S, int NT = stream_threads(S)>
__device__ __forceinline__ void spmm_gram2_body(const StepArgs<T>& a, int wg_id, int wg_cnt, double* red) {
  double acc[2 * S * S];
#pragma unroll
  for (int i = 0; i < 2 * S * S; ++i) acc[i] = 0.0;
  int lo, hi;
  op_rows(wg_id, wg_cnt, a.n, lo, hi);
  for (int r = lo + threadIdx.x; r < hi; r += NT) {
    T w[S], x[S], y[S];
    op_row<T, S>(a.op, a.Vcur, r, w);
    load_row<T, S>(a.Vprev + (size_t)r * S, x);
    load_row<T, S>(a.Vcur + (size_t)r * S, y);
    store_row<T, S>(a.W + (size_t)r * S, w);
#pragma unroll
    for (int p = 0; p < S; ++p)
#pragma unroll
      for (int q = 0; q < S; ++q) {
        acc[p * S + q] = fma((double)x[p], (double)w[q], acc[p * S + q]);
        acc[S * S + p * S + q] = fma((double)y[p], (double)w[q], acc[S * S + p * S + q]);
      }
  }
  write_partial_at<2 * S * S, NT>(acc, red, a.pout, wg_id);
}

// K2 / K3 (CGS2): W -= V_{j-1} c1, W -= V_j c2 with (c1, c2) the totals of the
// previous partials (logged in slot1, slot2); then the partials
// [V_{j-1}, V_j]^T W (first sweep) or W^T W (LAST: for the QR that follows).
template <typename T, int S, bool LAST, int NT = stream_threads(S)>
__device__ __forceinline__ void upd2_gram_body(const StepArgs<T>& a, int slot1, int slot2, int wg_id, int wg_cnt,
                                               double* red) {
  constexpr int K = LAST ? S * S : 2 * S * S;
  double c1[S * S], c2[S * S];
  take_gram2<S, NT>(a.pin, a.nparts, red, c1, c2, a.log + slot1 * S * S, a.log + slot2 * S * S, wg_id == 0);
  double acc[K];
#pragma unroll
  for (int i = 0; i < K; ++i) acc[i] = 0.0;
  int lo, hi;
  op_rows(wg_id, wg_cnt, a.n, lo, hi);
  for (int r = lo + threadIdx.x; r < hi; r += NT) {
    T w[S], x[S], y[S];
    load_row<T, S>(a.W + (size_t)r * S, w);
    load_row<T, S>(a.Vprev + (size_t)r * S, x);
    load_row<T, S>(a.Vcur + (size_t)r * S, y);
    upd_row<T, S>(w, x, c1);
    upd_row<T, S>(w, y, c2);
    store_row<T, S>(a.W + (size_t)r * S, w);
    if constexpr (LAST) {
      outer_acc<T, T, S>(acc, w, w);
    } else {
#pragma unroll
      for (int p = 0; p < S; ++p)
#pragma unroll
        for (int q = 0; q < S; ++q) {
          acc[p * S + q] = fma((double)x[p], (double)w[q], acc[p * S + q]);
          acc[S * S + p * S + q] = fma((double)y[p], (double)w[q], acc[S * S + p * S + q]);
        }
    }
  }
  write_partial_at<K, NT>(acc, red, a.pout, wg_id);
}

// K6: G1 = W^T W (logged), R1 = chol(G1) ; partial (W R1^{-1})^T (W R1^{-1})
template <typename T, int S, int NT = stream_threads(S)>
__device__ __forceinline__ void chol_gram_body(const StepArgs<T>& a, int wg_id, int wg_cnt, double* red) {
  __shared__ double sR1[S * S], sR1I[S * S];
  __shared__ double sratio;
  double G[S * S];
  take_gram<S, NT>(a.pin, a.nparts, red, G, a.log + L_G1 * S * S, wg_id == 0);
  if (threadIdx.x == 0) {
    sratio = chol_upper<S>(G, sR1);
    inv_upper<S>(sR1, sR1I);
  }
  __syncthreads();
  if (wg_id == 0 && threadIdx.x < S * S) {
    a.log[L_R1 * S * S + threadIdx.x] = sR1[threadIdx.x];
    a.log[L_R1I * S * S + threadIdx.x] = sR1I[threadIdx.x];
  }
  if (wg_id == 0 && threadIdx.x == 0) {
    double tr = 0.0;
    for (int i = 0; i < S; ++i) tr += G[i * S + i];
    a.log[L_FLAG * S * S + 0] = sratio;
    a.log[L_FLAG * S * S + 1] = tr;
    if (!(sratio > kBreakdownRatio) && a.flags[0] == 0) a.flags[0] = a.j + 1;
    if (!(tr == tr) || tr > 1e300) a.flags[1] = a.j + 1;
  }
  double ri[S * S];
#pragma unroll
  for (int i = 0; i < S * S; ++i) ri[i] = uniform_d(sR1I[i]);
  double acc[S * S];
  zero<S>(acc);
  const int str = wg_cnt * NT;
  LYAP_BATCH(r0, a.n) {
    T w[kRPT][S];
    LYAP_FOR_U {
      const int r = r0 + u * str;
      if (r < a.n) load_row<T, S>(a.W + (size_t)r * S, w[u]);
    }
    LYAP_FOR_U {
      const int r = r0 + u * str;
      if (r < a.n) {
        double uu[S];
        apply_upper_d<T, S>(w[u], ri, uu);
        outer_acc<double, double, S>(acc, uu, uu);
      }
    }
  }
  write_partial_at<S * S, NT>(acc, red, a.pout, wg_id);
}

// K7: G2 (logged), R2 = chol(G2), tau_{j+1,j} = R2 R1, V_{j+1} = W (R1^{-1} R2^{-1});
// workgroup 0 writes the log and the T_m band (diagonal block sym(alpha2 +
// alpha4), sub-diagonal block tau_{j+1,j}).
template <typename T, int S, int NT = stream_threads(S)>
__device__ __forceinline__ void chol_store_body(const StepArgs<T>& a, int wg_id, int wg_cnt, double* red) {
  __shared__ double sRI[S * S];
  double G[S * S];
  take_gram<S, NT>(a.pin, a.nparts, red, G, a.log + L_G2 * S * S, wg_id == 0);
  if (threadIdx.x == 0) {
    double R2[S * S], R2i[S * S], R[S * S];
    const double ratio = chol_upper<S>(G, R2);
    inv_upper<S>(R2, R2i);
    const double* L = a.log;
    mul_upper<S>(L + L_R1I * S * S, R2i, sRI);
    if (wg_id == 0) {
      double* Lw = a.log;
      mul_upper<S>(R2, L + L_R1 * S * S, R);
      for (int i = 0; i < S * S; ++i) {
        Lw[L_R2 * S * S + i] = R2[i];
        Lw[L_R * S * S + i] = R[i];
        Lw[L_RI * S * S + i] = sRI[i];
      }
      if (!(ratio > kBreakdownRatio) && a.flags[0] == 0) a.flags[0] = a.j + 1;
      const int ld = S + 1;
      const int c0 = a.j * S;
      for (int p = 0; p < S; ++p)
        for (int q = 0; q <= p; ++q) {
          const double tpq = L[L_A2 * S * S + p * S + q] + L[L_A4 * S * S + p * S + q];
          const double tqp = L[L_A2 * S * S + q * S + p] + L[L_A4 * S * S + q * S + p];
          a.band[(size_t)(c0 + q) * ld + (p - q)] = 0.5 * (tpq + tqp);
        }
      for (int p = 0; p < S; ++p)
        for (int q = p; q < S; ++q) a.band[(size_t)(c0 + q) * ld + (S + p - q)] = R[p * S + q];
    }
  }
  __syncthreads();
  double ri[S * S];
#pragma unroll
  for (int i = 0; i < S * S; ++i) ri[i] = uniform_d(sRI[i]);
  const int str = wg_cnt * NT;
  LYAP_BATCH(r0, a.n) {
    T w[kRPT][S];
    LYAP_FOR_U {
      const int r = r0 + u * str;
      if (r < a.n) load_row<T, S>(a.W + (size_t)r * S, w[u]);
    }
    LYAP_FOR_U {
      const int r = r0 + u * str;
      if (r < a.n) {
        T v[S];
        apply_upper<T, S>(w[u], ri, v);
        store_row<T, S>(a.Vnext + (size_t)r * S, v);
      }
    }
  }
}

// Second pass: the whole step from the log, one kernel (V_{j+1} may alias V_{j-1}).
template <typename T, int S, int NT = stream_threads(S)>
__device__ __forceinline__ void replay_body(const OpDev<T>& op, int n, const T* Vprev, const T* Vcur, T* Vnext,
                                            const double* log, int wg_id, int wg_cnt) {
  double a1[S * S], a2[S * S], a3[S * S], a4[S * S], ri[S * S];
  load_coef<S>(log + L_A1 * S * S, a1);
  load_coef<S>(log + L_A2 * S * S, a2);
  load_coef<S>(log + L_A3 * S * S, a3);
  load_coef<S>(log + L_A4 * S * S, a4);
  load_coef<S>(log + L_RI * S * S, ri);
  int lo, hi;
  op_rows(wg_id, wg_cnt, n, lo, hi);
  for (int r = lo + threadIdx.x; r < hi; r += NT) {
    T w[S], x[S], y[S], v[S];
    op_row<T, S>(op, Vcur, r, w);
    load_row<T, S>(Vprev + (size_t)r * S, x);
    load_row<T, S>(Vcur + (size_t)r * S, y);
    upd_row<T, S>(w, x, a1);
    upd_row<T, S>(w, y, a2);
    upd_row<T, S>(w, x, a3);
    upd_row<T, S>(w, y, a4);
    apply_upper<T, S>(w, ri, v);
    store_row<T, S>(Vnext + (size_t)r * S, v);
  }
}

// ------------------------------------------------------------------ single-problem kernels
template <typename T, int S>
__global__ __launch_bounds__(stream_threads(S)) void k_spmm_gram(StepArgs<T> a) {
  __shared__ double red[pow2_at_least(S * S) * (stream_threads(S) / 64)];
  spmm_gram_body<T, S>(a, blockIdx.x, gridDim.x, red);
}

template <typename T, int S>
__global__ __launch_bounds__(stream_threads(S)) void k_upd_gram(StepArgs<T> a, const T* X, const T* Y, int slot_in) {
  __shared__ double red[pow2_at_least(S * S) * (stream_threads(S) / 64)];
  upd_gram_body<T, S>(a, X, Y, slot_in, blockIdx.x, gridDim.x, red);
}

template <typename T, int S>
__global__ __launch_bounds__(stream_threads(S)) void k_spmm_gram2(StepArgs<T> a) {
  __shared__ double red[pow2_at_least(2 * S * S) * (stream_threads(S) / 64)];
  spmm_gram2_body<T, S>(a, blockIdx.x, gridDim.x, red);
}

template <typename T, int S, bool LAST>
__global__ __launch_bounds__(stream_threads(S)) void k_upd2_gram(StepArgs<T> a, int slot1, int slot2) {
  __shared__ double red[pow2_at_least(2 * S * S) * (stream_threads(S) / 64)];
  upd2_gram_body<T, S, LAST>(a, slot1, slot2, blockIdx.x, gridDim.x, red);
}

template <typename T, int S>
__global__ __launch_bounds__(stream_threads(S)) void k_chol_gram(StepArgs<T> a) {
  __shared__ double red[pow2_at_least(S * S) * (stream_threads(S) / 64)];
  chol_gram_body<T, S>(a, blockIdx.x, gridDim.x, red);
}

template <typename T, int S>
__global__ __launch_bounds__(stream_threads(S)) void k_chol_store(StepArgs<T> a) {
  __shared__ double red[pow2_at_least(S * S) * (stream_threads(S) / 64)];
  chol_store_body<T, S>(a, blockIdx.x, gridDim.x, red);
}

template <typename T, int S>
__global__ __launch_bounds__(stream_threads(S)) void k_replay(OpDev<T> op, int n, const T* Vprev, const T* Vcur,
                                                              T* Vnext, const double* log) {
  replay_body<T, S>(op, n, Vprev, Vcur, Vnext, log, blockIdx.x, gridDim.x);
}

// ------------------------------------------------------------------ initial block: C = V_1 gamma
template <int S>
__device__ __forceinline__ void load_C(const double* C, int64_t ldc, int r, double (&c)[S]) {
#pragma unroll
  for (int q = 0; q < S; ++q) c[q] = C[(size_t)q * ldc + r];
}

template <int S>
__global__ __launch_bounds__(stream_threads(S)) void k_init_gram(const double* C, int64_t ldc, int n, double* pout) {
  __shared__ double red[pow2_at_least(S * S) * (stream_threads(S) / 64)];
  double acc[S * S];
  zero<S>(acc);
  LYAP_ROWS(r, n) {
    double c[S];
    load_C<S>(C, ldc, r, c);
    outer_acc<double, double, S>(acc, c, c);
  }
  write_partial<S * S, stream_threads(S)>(acc, red, pout);
}

template <int S>
__global__ __launch_bounds__(stream_threads(S)) void k_init_chol_gram(const double* C, int64_t ldc, int n, double* glog,
                                                            const double* pin, int nparts, double* pout, int* flags) {
  __shared__ double red[pow2_at_least(S * S) * (stream_threads(S) / 64)];
  __shared__ double sR1[S * S], sR1I[S * S];
  __shared__ double sratio;
  double G[S * S];
  take_gram<S>(pin, nparts, red, G, glog + L_G1 * S * S, blockIdx.x == 0);
  if (threadIdx.x == 0) {
    sratio = chol_upper<S>(G, sR1);
    inv_upper<S>(sR1, sR1I);
  }
  __syncthreads();
  if (blockIdx.x == 0 && threadIdx.x < S * S) {
    glog[L_R1 * S * S + threadIdx.x] = sR1[threadIdx.x];
    glog[L_R1I * S * S + threadIdx.x] = sR1I[threadIdx.x];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    double tr = 0.0;
    for (int i = 0; i < S; ++i) tr += G[i * S + i];
    glog[L_FLAG * S * S + 0] = sratio;
    glog[L_FLAG * S * S + 1] = tr;
    if (!(tr == tr) || tr > 1e300) flags[1] = -1;
    if (!(sratio > kBreakdownRatio)) flags[0] = -1;
  }
  double ri[S * S];
#pragma unroll
  for (int i = 0; i < S * S; ++i) ri[i] = uniform_d(sR1I[i]);
  double acc[S * S];
  zero<S>(acc);
  LYAP_ROWS(r, n) {
    double c[S], u[S];
    load_C<S>(C, ldc, r, c);
    apply_upper_d<double, S>(c, ri, u);
    outer_acc<double, double, S>(acc, u, u);
  }
  write_partial<S * S, stream_threads(S)>(acc, red, pout);
}

template <typename T, int S>
__device__ __forceinline__ void store_V1(const double* C, int64_t ldc, int n, const double (&ri)[S * S], T* V1) {
  LYAP_ROWS(r, n) {
    double c[S], u[S];
    load_C<S>(C, ldc, r, c);
    apply_upper_d<double, S>(c, ri, u);
    T v[S];
#pragma unroll
    for (int q = 0; q < S; ++q) v[q] = (T)u[q];
    store_row<T, S>(V1 + (size_t)r * S, v);
  }
}

// gamma = R2 R1 (the positive-diagonal QR factor of C), V_1 = C gamma^{-1}
template <typename T, int S>
__global__ __launch_bounds__(stream_threads(S)) void k_init_store(const double* C, int64_t ldc, int n, double* glog,
                                                        const double* pin, int nparts, T* V1, int* flags) {
  __shared__ double red[pow2_at_least(S * S) * (stream_threads(S) / 64)];
  __shared__ double sRI[S * S];
  double G[S * S];
  take_gram<S>(pin, nparts, red, G, glog + L_G2 * S * S, blockIdx.x == 0);
  if (threadIdx.x == 0) {
    double R2[S * S], R2i[S * S], R[S * S];
    const double ratio = chol_upper<S>(G, R2);
    inv_upper<S>(R2, R2i);
    mul_upper<S>(glog + L_R1I * S * S, R2i, sRI);
    if (blockIdx.x == 0) {
      mul_upper<S>(R2, glog + L_R1 * S * S, R);
      for (int i = 0; i < S * S; ++i) {
        glog[L_R2 * S * S + i] = R2[i];
        glog[L_R * S * S + i] = R[i];
        glog[L_RI * S * S + i] = sRI[i];
      }
      if (!(ratio > kBreakdownRatio)) flags[0] = -1;
    }
  }
  __syncthreads();
  double ri[S * S];
#pragma unroll
  for (int i = 0; i < S * S; ++i) ri[i] = uniform_d(sRI[i]);
  store_V1<T, S>(C, ldc, n, ri, V1);
}

// V_1 again from the logged gamma^{-1} (second pass): same arithmetic.
template <typename T, int S>
__global__ __launch_bounds__(stream_threads(S)) void k_init_apply(const double* C, int64_t ldc, int n, const double* glog,
                                                        T* V1) {
  double ri[S * S];
  load_coef<S>(glog + L_RI * S * S, ri);
  store_V1<T, S>(C, ldc, n, ri, V1);
}

// ------------------------------------------------------------------ Z accumulation
// Z[:, c] += sum_{b < nb} V_b M_{[b]}[:, c] for the blocks listed in bl
// (nb <= 64), i.e. Z (n x t, column-major) += [V_b ...] (n x nb*S) times
// Mrows (nb*S x t, row-major).  Plain FP64 FMAs, accumulated in the order of
// the buffered blocks, starting from Z.  The work is FP64 FMA bound (2 nb S t
// flops per row against 16 t bytes of Z), so the tile is built for FMA issue
// and latency hiding: a lane owns zflush_rt rows (r, r + 64, ...) by kZCW
// columns of Z in registers (few enough registers for four or five waves per
// SIMD); the M row of a q-step, the same for the whole wave, is read with
// ordinary vector loads three q-steps ahead into a ring of four rows (vector
// loads return in order, so only the oldest is waited for; scalar loads
// would have to be waited for all together), and the rows of the next U
// blocks of V are loaded while the current ones are used (U blocks per
// iteration keep every q-step's ring slot static).  A workgroup's waves
// (blockDim / 64 of them) cover consecutive tiles of kZCW columns over the
// same rows, so V is read from HBM once per workgroup.  FULL: all kZCW
// columns of the wave exist; the last partial column tile runs as a separate
// launch with FULL = false (its columns past t read column t - 1 and are not
// stored).
constexpr int kZCW = 8, kZW = 8, kZRing = 4;
// blocks per iteration: the smallest U with U * S a multiple of the ring
constexpr int zflush_u(int S) {
  return S % 4 == 0 ? 1 : (S % 2 == 0 ? 2 : 4);
}
// rows per lane: at most 4, and the V rows of U blocks (twice: current and
// next) within 64 registers
template <typename T, int S>
constexpr int zflush_rt() {
  constexpr int regs = zflush_u(S) * S * (int)sizeof(T) / 4;  // per row
  return 32 / regs >= 4 ? 4 : (32 / regs >= 2 ? 2 : 1);
}

template <typename T, int S, bool FULL>
__global__ __launch_bounds__(64 * kZW) void k_zflush(BlockList bl, int nb, int n, const double* __restrict__ Mrows,
                                                     int ldm, int t, double* __restrict__ Z, int64_t ldz, int ncg) {
  constexpr int RT = zflush_rt<T, S>();
  constexpr int kZR = 64 * RT;
  constexpr int U = zflush_u(S);
  constexpr int R = kZRing, PD = kZRing - 1;
  static_assert((U * S) % R == 0, "every q-step's ring slot is static");
  // FULL: a 1-D launch over (row block, column group) pairs, dealt so that
  // each XCD takes a contiguous run of pairs: the ncg column groups of a row
  // block run back to back on one XCD, and all but the first read their rows
  // of V from that XCD's L2 rather than from HBM
  int rb = blockIdx.x, cg = 0;
  if constexpr (FULL) {
    const int lb = xcd_block(blockIdx.x, (int)((n + kZR - 1) / kZR) * ncg);
    if (lb < 0) return;
    rb = lb / ncg;
    cg = lb % ncg;
  }
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int nw = blockDim.x >> 6;
  const int c0 = (cg * nw + wv) * kZCW;
  if (c0 >= t) return;
  const int cmax = FULL ? kZCW - 1 : min(kZCW, t - c0) - 1;
  const int r0 = rb * kZR + lane;
  // rows past n compute on row n-1 (branch-free loads) and are not stored
  int rr[RT];
#pragma unroll
  for (int i = 0; i < RT; ++i) rr[i] = min(r0 + 64 * i, n - 1);
  double acc[RT][kZCW];
#pragma unroll
  for (int i = 0; i < RT; ++i)
#pragma unroll
    for (int c = 0; c < kZCW; ++c) acc[i][c] = Z[(size_t)(c0 + min(c, cmax)) * ldz + rr[i]];
  const int nq = nb * S;
  double mr[R][kZCW];
  auto loadm = [&](int qq, double (&dst)[kZCW]) {
    const double* src = Mrows + (size_t)min(qq, nq - 1) * ldm + c0;
#pragma unroll
    for (int c = 0; c < kZCW; ++c) dst[c] = src[FULL ? c : min(c, cmax)];
  };
#pragma unroll
  for (int d = 0; d < PD; ++d) loadm(d, mr[d]);
  T xs[U][RT][S];
#pragma unroll
  for (int u = 0; u < U; ++u)
#pragma unroll
    for (int i = 0; i < RT; ++i) load_row<T, S>((const T*)bl.p[min(u, nb - 1)] + (size_t)rr[i] * S, xs[u][i]);
#pragma unroll 1
  for (int b = 0; b < nb; b += U) {
    T xn[U][RT][S];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const T* Vn = (const T*)bl.p[min(b + U + u, nb - 1)];
#pragma unroll
      for (int i = 0; i < RT; ++i) load_row<T, S>(Vn + (size_t)rr[i] * S, xn[u][i]);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const bool live = b + u < nb;  // (uniform) the last group may be partial
#pragma unroll
      for (int q = 0; q < S; ++q) {
        const int ql = u * S + q;
        loadm((b + u) * S + q + PD, mr[(ql + PD) % R]);
        if (live) {
          const double(&cur)[kZCW] = mr[ql % R];
#pragma unroll
          for (int i = 0; i < RT; ++i) {
            const double a = (double)xs[u][i][q];
#pragma unroll
            for (int c = 0; c < kZCW; ++c) acc[i][c] = fma(a, cur[c], acc[i][c]);
          }
        }
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int i = 0; i < RT; ++i)
#pragma unroll
        for (int q = 0; q < S; ++q) xs[u][i][q] = xn[u][i][q];
  }
#pragma unroll
  for (int i = 0; i < RT; ++i) {
    const int r = r0 + 64 * i;
    if (r < n) {
#pragma unroll
      for (int c = 0; c < kZCW; ++c)
        if (c <= cmax) Z[(size_t)(c0 + c) * ldz + r] = acc[i][c];
    }
  }
}

template <typename T, int S>
__global__ __launch_bounds__(kBlock) void k_apply(OpDev<T> op, const T* V, T* W) {
  int lo, hi;
  op_rows(blockIdx.x, gridDim.x, op.n, lo, hi);
  for (int r = lo + threadIdx.x; r < hi; r += kBlock) {
    T w[S];
    op_row<T, S>(op, V, r, w);
    store_row_nt<T, S>(W + (size_t)r * S, w);
  }
}

// ------------------------------------------------------------------ grouped kernels
template <typename T, int S>
__device__ __forceinline__ StepArgs<T> batch_args(const BatchDesc<T>& d, int j, bool flip) {
  StepArgs<T> a{};
  a.op = d.op;
  a.n = d.n;
  const bool even = (j % 2) == 0;
  a.Vcur = even ? d.Vb1 : d.Vb0;
  T* other = even ? d.Vb0 : d.Vb1;
  a.Vprev = other;
  a.Vnext = other;
  a.W = d.W;
  a.log = d.log + (size_t)j * log_stride(S);
  a.band = d.band;
  a.j = j;
  a.pin = flip ? d.partA : d.partB;
  a.pout = flip ? d.partB : d.partA;
  a.nparts = d.nparts;
  a.flags = d.flags;
  return a;
}

template <typename T, int S, int NT>
__global__ __launch_bounds__(NT) void kb_spmm_gram(const BatchDesc<T>* __restrict__ d, const int2* __restrict__ map, const int* jp, int j) {
  __shared__ double red[pow2_at_least(S * S) * (NT / 64)];
  const int2 pm = map[blockIdx.x];
  if (jp) j = *jp;  // the step index held on the device (replayed graphs)
  const StepArgs<T> a = batch_args<T, S>(d[pm.x], j, false);
  spmm_gram_body<T, S, NT>(a, pm.y, a.nparts, red);
}

// mode 0: X = V_{j-1}, Y = V_j; 1: X = V_j, Y = V_{j-1}; 2: as 0; 3: X = V_j, Y = none
template <typename T, int S, int NT>
__global__ __launch_bounds__(NT) void kb_upd_gram(const BatchDesc<T>* __restrict__ d, const int2* __restrict__ map, const int* jp, int j,
                                                                 int mode, int slot, int flip) {
  __shared__ double red[pow2_at_least(S * S) * (NT / 64)];
  const int2 pm = map[blockIdx.x];
  if (jp) j = *jp;  // the step index held on the device (replayed graphs)
  const StepArgs<T> a = batch_args<T, S>(d[pm.x], j, flip != 0);
  const T* X = (mode == 0 || mode == 2) ? a.Vprev : a.Vcur;
  const T* Y = mode == 3 ? nullptr : ((mode == 1) ? a.Vprev : a.Vcur);
  upd_gram_body<T, S, NT>(a, X, Y, slot, pm.y, a.nparts, red);
}

template <typename T, int S, int NT>
__global__ __launch_bounds__(NT) void kb_spmm_gram2(const BatchDesc<T>* __restrict__ d, const int2* __restrict__ map, const int* jp, int j) {
  __shared__ double red[pow2_at_least(2 * S * S) * (NT / 64)];
  const int2 pm = map[blockIdx.x];
  if (jp) j = *jp;  // the step index held on the device (replayed graphs)
  const StepArgs<T> a = batch_args<T, S>(d[pm.x], j, false);
  spmm_gram2_body<T, S, NT>(a, pm.y, a.nparts, red);
}

template <typename T, int S, bool LAST, int NT>
__global__ __launch_bounds__(NT) void kb_upd2_gram(const BatchDesc<T>* __restrict__ d, const int2* __restrict__ map, const int* jp, int j,
                                                  int slot1, int slot2, int flip) {
  __shared__ double red[pow2_at_least(2 * S * S) * (NT / 64)];
  const int2 pm = map[blockIdx.x];
  if (jp) j = *jp;  // the step index held on the device (replayed graphs)
  const StepArgs<T> a = batch_args<T, S>(d[pm.x], j, flip != 0);
  upd2_gram_body<T, S, LAST, NT>(a, slot1, slot2, pm.y, a.nparts, red);
}

template <typename T, int S, int NT>
__global__ __launch_bounds__(NT) void kb_chol_gram(const BatchDesc<T>* __restrict__ d, const int2* __restrict__ map, const int* jp, int j) {
  __shared__ double red[pow2_at_least(S * S) * (NT / 64)];
  const int2 pm = map[blockIdx.x];
  if (jp) j = *jp;  // the step index held on the device (replayed graphs)
  const StepArgs<T> a = batch_args<T, S>(d[pm.x], j, true);
  chol_gram_body<T, S, NT>(a, pm.y, a.nparts, red);
}

template <typename T, int S, int NT>
__global__ __launch_bounds__(NT) void kb_chol_store(const BatchDesc<T>* __restrict__ d, const int2* __restrict__ map, const int* jp, int j) {
  __shared__ double red[pow2_at_least(S * S) * (NT / 64)];
  const int2 pm = map[blockIdx.x];
  if (jp) j = *jp;  // the step index held on the device (replayed graphs)
  const StepArgs<T> a = batch_args<T, S>(d[pm.x], j, false);
  chol_store_body<T, S, NT>(a, pm.y, a.nparts, red);
}

// Second pass step i of every problem in the map: V_{i+1} from V_i, V_{i-1}
// and log entry i, in the problem's ring of R blocks.
template <typename T, int S, int NT>
__global__ __launch_bounds__(NT) void kb_replay(const BatchDesc<T>* __restrict__ d, const int2* __restrict__ map, int i) {
  const int2 pm = map[blockIdx.x];
  const BatchDesc<T>& b = d[pm.x];
  const size_t nS = (size_t)b.n * S;
  const T* Vprev = i > 0 ? b.ring + (size_t)((i - 1) % b.R) * nS : b.zero;
  const T* Vcur = b.ring + (size_t)(i % b.R) * nS;
  T* Vnext = b.ring + (size_t)((i + 1) % b.R) * nS;
  replay_body<T, S, NT>(b.op, b.n, Vprev, Vcur, Vnext, b.log + (size_t)i * log_stride(S), pm.y, b.nparts);
}

// ------------------------------------------------------------------ host launchers
#define LYAP_SWITCH_S(Sv, ...)                                  \
  switch (Sv) {                                                 \
    case 1: { constexpr int S = 1; __VA_ARGS__; } break;        \
    case 2: { constexpr int S = 2; __VA_ARGS__; } break;        \
    case 3: { constexpr int S = 3; __VA_ARGS__; } break;        \
    case 4: { constexpr int S = 4; __VA_ARGS__; } break;        \
    case 5: { constexpr int S = 5; __VA_ARGS__; } break;        \
    case 6: { constexpr int S = 6; __VA_ARGS__; } break;        \
    case 7: { constexpr int S = 7; __VA_ARGS__; } break;        \
    case 8: { constexpr int S = 8; __VA_ARGS__; } break;        \
    default: LYAP_REQUIRE(false, LYAP_E_UNSUPPORTED, "block size %d not built", Sv); \
  }

template <typename T>
void launch_step(const StepArgs<T>& a0, int S, int grid, double* partA, double* partB, hipStream_t st,
                 KernelTimer* kt) {
  StepArgs<T> a = a0;
  a.nparts = grid;
  auto mark = [&](int k) { if (kt) kt->mark(k); };
  LYAP_SWITCH_S(S, {
    if constexpr (cgs2_width(S)) {
      a.pin = nullptr; a.pout = partA;
      mark(LYAP_K_SPMM_GRAM);
      hipLaunchKernelGGL((k_spmm_gram2<T, S>), dim3(grid), dim3(stream_threads(S)), 0, st, a);
      a.pin = partA; a.pout = partB;
      mark(LYAP_K_UPD_GRAM);
      hipLaunchKernelGGL((k_upd2_gram<T, S, false>), dim3(grid), dim3(stream_threads(S)), 0, st, a, (int)L_A1,
                         (int)L_A2);
      a.pin = partB; a.pout = partA;
      mark(LYAP_K_UPD_GRAM);
      hipLaunchKernelGGL((k_upd2_gram<T, S, true>), dim3(grid), dim3(stream_threads(S)), 0, st, a, (int)L_A3,
                         (int)L_A4);
      a.pin = partA; a.pout = partB;
      mark(LYAP_K_CHOL_GRAM);
      hipLaunchKernelGGL((k_chol_gram<T, S>), dim3(grid), dim3(stream_threads(S)), 0, st, a);
      a.pin = partB; a.pout = partA;
      mark(LYAP_K_CHOL_STORE);
      hipLaunchKernelGGL((k_chol_store<T, S>), dim3(grid), dim3(stream_threads(S)), 0, st, a);
    } else {
      a.pin = nullptr; a.pout = partA;
      mark(LYAP_K_SPMM_GRAM);
      hipLaunchKernelGGL((k_spmm_gram<T, S>), dim3(grid), dim3(stream_threads(S)), 0, st, a);
      a.pin = partA; a.pout = partB;
      mark(LYAP_K_UPD_GRAM);
      hipLaunchKernelGGL((k_upd_gram<T, S>), dim3(grid), dim3(stream_threads(S)), 0, st, a, a.Vprev, a.Vcur, (int)L_A1);
      a.pin = partB; a.pout = partA;
      mark(LYAP_K_UPD_GRAM);
      hipLaunchKernelGGL((k_upd_gram<T, S>), dim3(grid), dim3(stream_threads(S)), 0, st, a, a.Vcur, a.Vprev, (int)L_A2);
      a.pin = partA; a.pout = partB;
      mark(LYAP_K_UPD_GRAM);
      hipLaunchKernelGGL((k_upd_gram<T, S>), dim3(grid), dim3(stream_threads(S)), 0, st, a, a.Vprev, a.Vcur, (int)L_A3);
      a.pin = partB; a.pout = partA;
      mark(LYAP_K_UPD_GRAM);
      hipLaunchKernelGGL((k_upd_gram<T, S>), dim3(grid), dim3(stream_threads(S)), 0, st, a, a.Vcur, (const T*)nullptr, (int)L_A4);
      a.pin = partA; a.pout = partB;
      mark(LYAP_K_CHOL_GRAM);
      hipLaunchKernelGGL((k_chol_gram<T, S>), dim3(grid), dim3(stream_threads(S)), 0, st, a);
      a.pin = partB; a.pout = partA;
      mark(LYAP_K_CHOL_STORE);
      hipLaunchKernelGGL((k_chol_store<T, S>), dim3(grid), dim3(stream_threads(S)), 0, st, a);
    }
  });
  LYAP_LAUNCHED("lanczos step");
}

template <typename T>
void launch_replay(const OpDev<T>& op, int S, const T* Vprev, const T* Vcur, T* Vnext, const double* log, int grid,
                   hipStream_t st) {
  LYAP_SWITCH_S(S, { hipLaunchKernelGGL((k_replay<T, S>), dim3(grid), dim3(stream_threads(S)), 0, st, op, op.n, Vprev, Vcur, Vnext, log); });
  LYAP_LAUNCHED("replay");
}

template <typename T>
void launch_init(const double* C, int64_t ldc, int n, int S, double* glog, double* partA, double* partB, int* flags,
                 T* V1, int grid, hipStream_t st) {
  LYAP_SWITCH_S(S, {
    hipLaunchKernelGGL((k_init_gram<S>), dim3(grid), dim3(stream_threads(S)), 0, st, C, ldc, n, partA);
    hipLaunchKernelGGL((k_init_chol_gram<S>), dim3(grid), dim3(stream_threads(S)), 0, st, C, ldc, n, glog, partA, grid, partB,
                       flags);
    hipLaunchKernelGGL((k_init_store<T, S>), dim3(grid), dim3(stream_threads(S)), 0, st, C, ldc, n, glog, partB, grid, V1, flags);
  });
  LYAP_LAUNCHED("init");
}

template <typename T>
void launch_init_store(const double* C, int64_t ldc, int n, int S, const double* glog, T* V1, int grid, hipStream_t st) {
  LYAP_SWITCH_S(S, { hipLaunchKernelGGL((k_init_apply<T, S>), dim3(grid), dim3(stream_threads(S)), 0, st, C, ldc, n, glog, V1); });
  LYAP_LAUNCHED("init_apply");
}

template <typename T>
void launch_zflush(const void* const* blocks, int nb, int n, int S, const double* Mrows, int t, double* Z,
                   int64_t ldz, int /*grid*/, hipStream_t st) {
  if (nb <= 0 || t <= 0) return;
  LYAP_SWITCH_S(S, {
    int done = 0;
    while (done < nb) {
      const int cnt = nb - done < 64 ? nb - done : 64;
      BlockList bl{};
      for (int b = 0; b < cnt; ++b) bl.p[b] = blocks[done + b];
      const double* Mc = Mrows + (size_t)done * S * t;
      const int tf = t / kZCW * kZCW;  // columns in full tiles
      constexpr int kZR = 64 * zflush_rt<T, S>();
      if (tf > 0) {
        // column groups of at most kZW tiles, the tiles spread evenly over them
        const int tiles = tf / kZCW;
        const int ncg = (tiles + kZW - 1) / kZW;
        const int nw = (tiles + ncg - 1) / ncg;  // waves per workgroup
        const int pairs = (n + kZR - 1) / kZR * ncg;
        hipLaunchKernelGGL((k_zflush<T, S, true>), dim3(xcd_grid(pairs)), dim3(64 * nw), 0, st, bl, cnt, n, Mc, t,
                           tf, Z, ldz, ncg);
      }
      if (tf < t)
        hipLaunchKernelGGL((k_zflush<T, S, false>), dim3((n + kZR - 1) / kZR, 1), dim3(64), 0, st, bl, cnt, n, Mc + tf,
                           t, t - tf, Z + (size_t)tf * ldz, ldz, 1);
      done += cnt;
    }
  });
  LYAP_LAUNCHED("zflush");
}

int zflush_max_blocks(int) { return 64; }

// Grouped launches with nt threads per workgroup: 256 or 1024 for blocks of
// at most 4 columns (the autotuner's choice), 256 above (register budget).
#define LYAP_SWITCH_NT(S, ntv, ...)                                              \
  if ((S) <= 4 && (ntv) == 1024) {                                               \
    constexpr int NT = 1024;                                                     \
    __VA_ARGS__;                                                                 \
  } else {                                                                       \
    LYAP_REQUIRE((ntv) == 256 || ((ntv) == 1024 && (S) > 4), LYAP_E_ARG,         \
                 "workgroup size %d not built for block width %d", (ntv), (S));  \
    constexpr int NT = 256;                                                      \
    __VA_ARGS__;                                                                 \
  }

int batch_default_threads(int S) { return stream_threads(S); }

template <typename T>
void launch_batch_step(const BatchDesc<T>* d, const int2* map, int nwg, int S, int nt, int j, hipStream_t st,
                       KernelTimer* kt, const int* jp) {
  if (nwg <= 0) return;
  auto mark = [&](int k) { if (kt) kt->mark(k); };
  LYAP_SWITCH_S(S, {
    LYAP_SWITCH_NT(S, nt, {
      if constexpr (cgs2_width(S)) {
        mark(LYAP_K_SPMM_GRAM);
        hipLaunchKernelGGL((kb_spmm_gram2<T, S, NT>), dim3(nwg), dim3(NT), 0, st, d, map, jp, j);
        mark(LYAP_K_UPD_GRAM);
        hipLaunchKernelGGL((kb_upd2_gram<T, S, false, NT>), dim3(nwg), dim3(NT), 0, st, d, map, jp, j, (int)L_A1,
                           (int)L_A2, 1);
        mark(LYAP_K_UPD_GRAM);
        hipLaunchKernelGGL((kb_upd2_gram<T, S, true, NT>), dim3(nwg), dim3(NT), 0, st, d, map, jp, j, (int)L_A3,
                           (int)L_A4, 0);
        mark(LYAP_K_CHOL_GRAM);
        hipLaunchKernelGGL((kb_chol_gram<T, S, NT>), dim3(nwg), dim3(NT), 0, st, d, map, jp, j);
        mark(LYAP_K_CHOL_STORE);
        hipLaunchKernelGGL((kb_chol_store<T, S, NT>), dim3(nwg), dim3(NT), 0, st, d, map, jp, j);
      } else {
        mark(LYAP_K_SPMM_GRAM);
        hipLaunchKernelGGL((kb_spmm_gram<T, S, NT>), dim3(nwg), dim3(NT), 0, st, d, map, jp, j);
        mark(LYAP_K_UPD_GRAM);
        hipLaunchKernelGGL((kb_upd_gram<T, S, NT>), dim3(nwg), dim3(NT), 0, st, d, map, jp, j, 0, (int)L_A1, 1);
        mark(LYAP_K_UPD_GRAM);
        hipLaunchKernelGGL((kb_upd_gram<T, S, NT>), dim3(nwg), dim3(NT), 0, st, d, map, jp, j, 1, (int)L_A2, 0);
        mark(LYAP_K_UPD_GRAM);
        hipLaunchKernelGGL((kb_upd_gram<T, S, NT>), dim3(nwg), dim3(NT), 0, st, d, map, jp, j, 2, (int)L_A3, 1);
        mark(LYAP_K_UPD_GRAM);
        hipLaunchKernelGGL((kb_upd_gram<T, S, NT>), dim3(nwg), dim3(NT), 0, st, d, map, jp, j, 3, (int)L_A4, 0);
        mark(LYAP_K_CHOL_GRAM);
        hipLaunchKernelGGL((kb_chol_gram<T, S, NT>), dim3(nwg), dim3(NT), 0, st, d, map, jp, j);
        mark(LYAP_K_CHOL_STORE);
        hipLaunchKernelGGL((kb_chol_store<T, S, NT>), dim3(nwg), dim3(NT), 0, st, d, map, jp, j);
      }
    });
  });
  LYAP_LAUNCHED("batched lanczos step");
}

template <typename T>
void launch_batch_replay(const BatchDesc<T>* d, const int2* map, int nwg, int S, int nt, int i, hipStream_t st) {
  if (nwg <= 0) return;
  LYAP_SWITCH_S(S, {
    LYAP_SWITCH_NT(S, nt, { hipLaunchKernelGGL((kb_replay<T, S, NT>), dim3(nwg), dim3(NT), 0, st, d, map, i); });
  });
  LYAP_LAUNCHED("batched replay");
}

template <typename T>
void launch_apply(const OpDev<T>& op, int S, const T* V, T* W, int grid, hipStream_t st) {
  LYAP_SWITCH_S(S, { hipLaunchKernelGGL((k_apply<T, S>), dim3(grid), dim3(kBlock), 0, st, op, V, W); });
  LYAP_LAUNCHED("apply");
}

#define LYAP_INST(T)                                                                                         \
  template void launch_step<T>(const StepArgs<T>&, int, int, double*, double*, hipStream_t, KernelTimer*);  \
  template void launch_replay<T>(const OpDev<T>&, int, const T*, const T*, T*, const double*, int, hipStream_t); \
  template void launch_init<T>(const double*, int64_t, int, int, double*, double*, double*, int*, T*, int,     \
                               hipStream_t);                                                                 \
  template void launch_init_store<T>(const double*, int64_t, int, int, const double*, T*, int, hipStream_t);  \
  template void launch_zflush<T>(const void* const*, int, int, int, const double*, int, double*, int64_t, int, \
                                 hipStream_t);                                                               \
  template void launch_apply<T>(const OpDev<T>&, int, const T*, T*, int, hipStream_t);                     \
  template void launch_batch_step<T>(const BatchDesc<T>*, const int2*, int, int, int, int, hipStream_t,          \
                                     KernelTimer*, const int*);                                                \
  template void launch_batch_replay<T>(const BatchDesc<T>*, const int2*, int, int, int, int, hipStream_t);

LYAP_INST(float)
LYAP_INST(double)

}  // namespace lyap

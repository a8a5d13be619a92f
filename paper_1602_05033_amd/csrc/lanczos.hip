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
#pragma unroll
  for (int i = 0; i < S * S; ++i) dst[i] = src[i];
}

// ------------------------------------------------------------------ small dense FP64 helpers
// G = R^T R, R upper triangular with positive diagonal.  Returns the smallest
// pivot ratio d_i / G_ii (1 = orthogonal columns, 0 = dependent).
template <int S>
__device__ double chol_upper(const double* G, double* R) {
  double ratio = 1.0;
  for (int i = 0; i < S; ++i)
    for (int j = 0; j < S; ++j) R[i * S + j] = 0.0;
  for (int i = 0; i < S; ++i) {
    double d = G[i * S + i];
    for (int k = 0; k < i; ++k) d -= R[k * S + i] * R[k * S + i];
    const double gi = G[i * S + i];
    const double r = gi > 0.0 ? d / gi : 0.0;
    if (!(r >= 0.0)) ratio = 0.0;
    else if (r < ratio) ratio = r;
    const double dd = d > 1e-300 ? d : 1e-300;
    const double rii = sqrt(dd);
    R[i * S + i] = rii;
    for (int j = i + 1; j < S; ++j) {
      double v = G[i * S + j];
      for (int k = 0; k < i; ++k) v -= R[k * S + i] * R[k * S + j];
      R[i * S + j] = v / rii;
    }
  }
  return ratio;
}

template <int S>
__device__ void inv_upper(const double* R, double* Ri) {
  for (int i = 0; i < S * S; ++i) Ri[i] = 0.0;
  for (int j = 0; j < S; ++j) {
    Ri[j * S + j] = 1.0 / R[j * S + j];
    for (int i = j - 1; i >= 0; --i) {
      double acc = 0.0;
      for (int k = i; k < j; ++k) acc += Ri[i * S + k] * R[k * S + j];
      Ri[i * S + j] = -acc / R[j * S + j];
    }
  }
}

template <int S>
__device__ void mul_upper(const double* A, const double* B, double* C) {  // C = A B
  for (int i = 0; i < S; ++i)
    for (int j = 0; j < S; ++j) {
      double acc = 0.0;
      for (int k = 0; k < S; ++k) acc += A[i * S + k] * B[k * S + j];
      C[i * S + j] = acc;
    }
}

// breakdown when a Cholesky pivot keeps less than this fraction of the
// squared column norm (the block is numerically rank deficient)
constexpr double kBreakdownRatio = 1e-14;

// ------------------------------------------------------------------ kernels
// K1: W = A V_j ; alpha1 = V_{j-1}^T W
template <typename T, int S>
__global__ __launch_bounds__(kBlock) void k_spmm_gram(StepArgs<T> a) {
  __shared__ double red[S * S * kWaves];
  double acc[S * S];
#pragma unroll
  for (int i = 0; i < S * S; ++i) acc[i] = 0.0;
  for (int r = blockIdx.x * kBlock + threadIdx.x; r < a.n; r += gridDim.x * kBlock) {
    T w[S], x[S];
    op_row<T, S>(a.op, a.Vcur, r, w);
    store_row<T, S>(a.W + (size_t)r * S, w);
    load_row<T, S>(a.Vprev + (size_t)r * S, x);
#pragma unroll
    for (int p = 0; p < S; ++p)
#pragma unroll
      for (int q = 0; q < S; ++q) acc[p * S + q] = fma((double)x[p], (double)w[q], acc[p * S + q]);
  }
  if (grid_sum_last<S * S>(acc, red, a.part, a.counter)) {
    if (threadIdx.x < S * S) a.log[L_A1 * S * S + threadIdx.x] = red[threadIdx.x];
  }
}

// K2..K4: W -= X alpha_in ; alpha_out = Y^T W
template <typename T, int S>
__global__ __launch_bounds__(kBlock) void k_upd_gram(StepArgs<T> a, const T* X, const T* Y, int slot_in,
                                                     int slot_out) {
  __shared__ double red[S * S * kWaves];
  double al[S * S];
  load_coef<S>(a.log + slot_in * S * S, al);
  double acc[S * S];
#pragma unroll
  for (int i = 0; i < S * S; ++i) acc[i] = 0.0;
  for (int r = blockIdx.x * kBlock + threadIdx.x; r < a.n; r += gridDim.x * kBlock) {
    T w[S], x[S], y[S];
    load_row<T, S>(a.W + (size_t)r * S, w);
    load_row<T, S>(X + (size_t)r * S, x);
    upd_row<T, S>(w, x, al);
    store_row<T, S>(a.W + (size_t)r * S, w);
    load_row<T, S>(Y + (size_t)r * S, y);
#pragma unroll
    for (int p = 0; p < S; ++p)
#pragma unroll
      for (int q = 0; q < S; ++q) acc[p * S + q] = fma((double)y[p], (double)w[q], acc[p * S + q]);
  }
  if (grid_sum_last<S * S>(acc, red, a.part, a.counter)) {
    if (threadIdx.x < S * S) a.log[slot_out * S * S + threadIdx.x] = red[threadIdx.x];
  }
}

// K5: W -= V_j alpha4 ; G1 = W^T W ; R1 = chol(G1)
template <typename T, int S>
__global__ __launch_bounds__(kBlock) void k_upd_gramself(StepArgs<T> a) {
  __shared__ double red[S * S * kWaves];
  double al[S * S];
  load_coef<S>(a.log + L_A4 * S * S, al);
  double acc[S * S];
#pragma unroll
  for (int i = 0; i < S * S; ++i) acc[i] = 0.0;
  for (int r = blockIdx.x * kBlock + threadIdx.x; r < a.n; r += gridDim.x * kBlock) {
    T w[S], x[S];
    load_row<T, S>(a.W + (size_t)r * S, w);
    load_row<T, S>(a.Vcur + (size_t)r * S, x);
    upd_row<T, S>(w, x, al);
    store_row<T, S>(a.W + (size_t)r * S, w);
#pragma unroll
    for (int p = 0; p < S; ++p)
#pragma unroll
      for (int q = 0; q < S; ++q) acc[p * S + q] = fma((double)w[p], (double)w[q], acc[p * S + q]);
  }
  if (grid_sum_last<S * S>(acc, red, a.part, a.counter)) {
    if (threadIdx.x == 0) {
      double* L = a.log;
      for (int i = 0; i < S * S; ++i) L[L_G1 * S * S + i] = red[i];
      double ratio = chol_upper<S>(L + L_G1 * S * S, L + L_R1 * S * S);
      inv_upper<S>(L + L_R1 * S * S, L + L_R1I * S * S);
      double tr = 0.0;
      for (int i = 0; i < S; ++i) tr += red[i * S + i];
      L[L_FLAG * S * S + 0] = ratio;
      L[L_FLAG * S * S + 1] = tr;
      if (!(ratio > kBreakdownRatio) && a.flags[0] == 0) a.flags[0] = a.j + 1;
      if (!(tr == tr) || tr > 1e300) a.flags[1] = a.j + 1;
    }
  }
}

// K6: U = W R1^{-1} ; G2 = U^T U ; R2 = chol(G2) ; tau_{j+1,j} = R2 R1 ; T band
template <typename T, int S>
__global__ __launch_bounds__(kBlock) void k_apply_gramself(StepArgs<T> a) {
  __shared__ double red[S * S * kWaves];
  double ri[S * S];
  load_coef<S>(a.log + L_R1I * S * S, ri);
  double acc[S * S];
#pragma unroll
  for (int i = 0; i < S * S; ++i) acc[i] = 0.0;
  for (int r = blockIdx.x * kBlock + threadIdx.x; r < a.n; r += gridDim.x * kBlock) {
    T w[S];
    double u[S];
    load_row<T, S>(a.W + (size_t)r * S, w);
    apply_upper_d<T, S>(w, ri, u);
#pragma unroll
    for (int p = 0; p < S; ++p)
#pragma unroll
      for (int q = 0; q < S; ++q) acc[p * S + q] = fma(u[p], u[q], acc[p * S + q]);
  }
  if (grid_sum_last<S * S>(acc, red, a.part, a.counter)) {
    if (threadIdx.x == 0) {
      double* L = a.log;
      for (int i = 0; i < S * S; ++i) L[L_G2 * S * S + i] = red[i];
      double ratio = chol_upper<S>(L + L_G2 * S * S, L + L_R2 * S * S);
      double R2i[S * S];
      inv_upper<S>(L + L_R2 * S * S, R2i);
      mul_upper<S>(L + L_R2 * S * S, L + L_R1 * S * S, L + L_R * S * S);
      mul_upper<S>(L + L_R1I * S * S, R2i, L + L_RI * S * S);
      if (!(ratio > kBreakdownRatio) && a.flags[0] == 0) a.flags[0] = a.j + 1;
      // T_m band (lower, ld = S+1): diagonal block sym(alpha2 + alpha4),
      // sub-diagonal block tau_{j+1,j} = R.
      const int ld = S + 1;
      const int c0 = a.j * S;
      for (int p = 0; p < S; ++p)
        for (int q = 0; q <= p; ++q) {
          const double tpq = L[L_A2 * S * S + p * S + q] + L[L_A4 * S * S + p * S + q];
          const double tqp = L[L_A2 * S * S + q * S + p] + L[L_A4 * S * S + q * S + p];
          a.band[(size_t)(c0 + q) * ld + (p - q)] = 0.5 * (tpq + tqp);
        }
      for (int p = 0; p < S; ++p)
        for (int q = p; q < S; ++q) a.band[(size_t)(c0 + q) * ld + (S + p - q)] = L[L_R * S * S + p * S + q];
    }
  }
}

// K7: V_{j+1} = W (R1^{-1} R2^{-1})
template <typename T, int S>
__global__ __launch_bounds__(kBlock) void k_apply_store(StepArgs<T> a) {
  double ri[S * S];
  load_coef<S>(a.log + L_RI * S * S, ri);
  for (int r = blockIdx.x * kBlock + threadIdx.x; r < a.n; r += gridDim.x * kBlock) {
    T w[S], v[S];
    load_row<T, S>(a.W + (size_t)r * S, w);
    apply_upper<T, S>(w, ri, v);
    store_row<T, S>(a.Vnext + (size_t)r * S, v);
  }
}

// Second pass: the whole step from the log, one kernel (V_{j+1} may alias V_{j-1}).
template <typename T, int S>
__global__ __launch_bounds__(kBlock) void k_replay(OpDev<T> op, int n, const T* Vprev, const T* Vcur, T* Vnext,
                                                   const double* log) {
  double a1[S * S], a2[S * S], a3[S * S], a4[S * S], ri[S * S];
  load_coef<S>(log + L_A1 * S * S, a1);
  load_coef<S>(log + L_A2 * S * S, a2);
  load_coef<S>(log + L_A3 * S * S, a3);
  load_coef<S>(log + L_A4 * S * S, a4);
  load_coef<S>(log + L_RI * S * S, ri);
  for (int r = blockIdx.x * kBlock + threadIdx.x; r < n; r += gridDim.x * kBlock) {
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

// ------------------------------------------------------------------ initial block: C = V_1 gamma
template <int S>
__global__ __launch_bounds__(kBlock) void k_init_gram(const double* C, int64_t ldc, int n, double* glog,
                                                      double* part, unsigned* counter, int* flags) {
  __shared__ double red[S * S * kWaves];
  double acc[S * S];
#pragma unroll
  for (int i = 0; i < S * S; ++i) acc[i] = 0.0;
  for (int r = blockIdx.x * kBlock + threadIdx.x; r < n; r += gridDim.x * kBlock) {
    double c[S];
#pragma unroll
    for (int q = 0; q < S; ++q) c[q] = C[(size_t)q * ldc + r];
#pragma unroll
    for (int p = 0; p < S; ++p)
#pragma unroll
      for (int q = 0; q < S; ++q) acc[p * S + q] = fma(c[p], c[q], acc[p * S + q]);
  }
  if (grid_sum_last<S * S>(acc, red, part, counter)) {
    if (threadIdx.x == 0) {
      for (int i = 0; i < S * S; ++i) glog[L_G1 * S * S + i] = red[i];
      double tr = 0.0;
      for (int i = 0; i < S; ++i) tr += red[i * S + i];
      double ratio = chol_upper<S>(glog + L_G1 * S * S, glog + L_R1 * S * S);
      inv_upper<S>(glog + L_R1 * S * S, glog + L_R1I * S * S);
      glog[L_FLAG * S * S + 0] = ratio;
      glog[L_FLAG * S * S + 1] = tr;
      if (!(tr == tr) || tr > 1e300) flags[1] = -1;
      if (!(ratio > kBreakdownRatio)) flags[0] = -1;
    }
  }
}

template <int S>
__global__ __launch_bounds__(kBlock) void k_init_gram2(const double* C, int64_t ldc, int n, double* glog,
                                                       double* part, unsigned* counter, int* flags) {
  __shared__ double red[S * S * kWaves];
  double ri[S * S];
  load_coef<S>(glog + L_R1I * S * S, ri);
  double acc[S * S];
#pragma unroll
  for (int i = 0; i < S * S; ++i) acc[i] = 0.0;
  for (int r = blockIdx.x * kBlock + threadIdx.x; r < n; r += gridDim.x * kBlock) {
    double c[S], u[S];
#pragma unroll
    for (int q = 0; q < S; ++q) c[q] = C[(size_t)q * ldc + r];
    apply_upper_d<double, S>(c, ri, u);
#pragma unroll
    for (int p = 0; p < S; ++p)
#pragma unroll
      for (int q = 0; q < S; ++q) acc[p * S + q] = fma(u[p], u[q], acc[p * S + q]);
  }
  if (grid_sum_last<S * S>(acc, red, part, counter)) {
    if (threadIdx.x == 0) {
      for (int i = 0; i < S * S; ++i) glog[L_G2 * S * S + i] = red[i];
      double ratio = chol_upper<S>(glog + L_G2 * S * S, glog + L_R2 * S * S);
      double R2i[S * S];
      inv_upper<S>(glog + L_R2 * S * S, R2i);
      mul_upper<S>(glog + L_R2 * S * S, glog + L_R1 * S * S, glog + L_R * S * S);    // gamma
      mul_upper<S>(glog + L_R1I * S * S, R2i, glog + L_RI * S * S);                 // gamma^{-1}
      if (!(ratio > kBreakdownRatio)) flags[0] = -1;
    }
  }
}

template <typename T, int S>
__global__ __launch_bounds__(kBlock) void k_init_store(const double* C, int64_t ldc, int n, const double* glog,
                                                       T* V1) {
  double ri[S * S];
  load_coef<S>(glog + L_RI * S * S, ri);
  for (int r = blockIdx.x * kBlock + threadIdx.x; r < n; r += gridDim.x * kBlock) {
    double c[S], u[S];
#pragma unroll
    for (int q = 0; q < S; ++q) c[q] = C[(size_t)q * ldc + r];
    apply_upper_d<double, S>(c, ri, u);
    T v[S];
#pragma unroll
    for (int q = 0; q < S; ++q) v[q] = (T)u[q];
    store_row<T, S>(V1 + (size_t)r * S, v);
  }
}

// ------------------------------------------------------------------ Z accumulation
// Z[:, c] += sum_{b < nb} V_b M_{[b]}[:, c] for the blocks listed in bl.
// Mrows: row-major (nb*S) x t rows of M belonging to those blocks, in order.
template <typename T, int S>
__global__ __launch_bounds__(kBlock) void k_zflush(BlockList bl, int nb, int n, const double* Mrows, int t, double* Z,
                                                   int64_t ldz) {
  constexpr int QB = (64 / S) > 0 ? 64 / S : 1;
  for (int r = blockIdx.x * kBlock + threadIdx.x; r < n; r += gridDim.x * kBlock) {
    double v[QB * S];
#pragma unroll
    for (int b = 0; b < QB; ++b) {
      if (b < nb) {
        T x[S];
        load_row<T, S>((const T*)bl.p[b] + (size_t)r * S, x);
#pragma unroll
        for (int q = 0; q < S; ++q) v[b * S + q] = (double)x[q];
      } else {
#pragma unroll
        for (int q = 0; q < S; ++q) v[b * S + q] = 0.0;
      }
    }
    for (int c = 0; c < t; ++c) {
      double acc = Z[(size_t)c * ldz + r];
#pragma unroll
      for (int b = 0; b < QB; ++b) {
        if (b < nb) {
#pragma unroll
          for (int q = 0; q < S; ++q) acc = fma(v[b * S + q], Mrows[(size_t)(b * S + q) * t + c], acc);
        }
      }
      Z[(size_t)c * ldz + r] = acc;
    }
  }
}

template <typename T, int S>
__global__ __launch_bounds__(kBlock) void k_apply(OpDev<T> op, const T* V, T* W) {
  for (int r = blockIdx.x * kBlock + threadIdx.x; r < op.n; r += gridDim.x * kBlock) {
    T w[S];
    op_row<T, S>(op, V, r, w);
    store_row<T, S>(W + (size_t)r * S, w);
  }
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
void launch_step(const StepArgs<T>& a, int S, int grid, hipStream_t st) {
  LYAP_SWITCH_S(S, {
    hipLaunchKernelGGL((k_spmm_gram<T, S>), dim3(grid), dim3(kBlock), 0, st, a);
    hipLaunchKernelGGL((k_upd_gram<T, S>), dim3(grid), dim3(kBlock), 0, st, a, a.Vprev, a.Vcur, (int)L_A1, (int)L_A2);
    hipLaunchKernelGGL((k_upd_gram<T, S>), dim3(grid), dim3(kBlock), 0, st, a, a.Vcur, a.Vprev, (int)L_A2, (int)L_A3);
    hipLaunchKernelGGL((k_upd_gram<T, S>), dim3(grid), dim3(kBlock), 0, st, a, a.Vprev, a.Vcur, (int)L_A3, (int)L_A4);
    hipLaunchKernelGGL((k_upd_gramself<T, S>), dim3(grid), dim3(kBlock), 0, st, a);
    hipLaunchKernelGGL((k_apply_gramself<T, S>), dim3(grid), dim3(kBlock), 0, st, a);
    hipLaunchKernelGGL((k_apply_store<T, S>), dim3(grid), dim3(kBlock), 0, st, a);
  });
  LYAP_LAUNCHED("lanczos step");
}

template <typename T>
void launch_replay(const OpDev<T>& op, int S, const T* Vprev, const T* Vcur, T* Vnext, const double* log, int grid,
                   hipStream_t st) {
  LYAP_SWITCH_S(S, { hipLaunchKernelGGL((k_replay<T, S>), dim3(grid), dim3(kBlock), 0, st, op, op.n, Vprev, Vcur, Vnext, log); });
  LYAP_LAUNCHED("replay");
}

template <typename T>
void launch_init(const double* C, int64_t ldc, int n, int S, double* glog, double* part, unsigned* counter, int* flags,
                 T* V1, int grid, hipStream_t st) {
  LYAP_SWITCH_S(S, {
    hipLaunchKernelGGL((k_init_gram<S>), dim3(grid), dim3(kBlock), 0, st, C, ldc, n, glog, part, counter, flags);
    hipLaunchKernelGGL((k_init_gram2<S>), dim3(grid), dim3(kBlock), 0, st, C, ldc, n, glog, part, counter, flags);
    hipLaunchKernelGGL((k_init_store<T, S>), dim3(grid), dim3(kBlock), 0, st, C, ldc, n, glog, V1);
  });
  LYAP_LAUNCHED("init");
}

template <typename T>
void launch_init_store(const double* C, int64_t ldc, int n, int S, const double* glog, T* V1, int grid, hipStream_t st) {
  LYAP_SWITCH_S(S, { hipLaunchKernelGGL((k_init_store<T, S>), dim3(grid), dim3(kBlock), 0, st, C, ldc, n, glog, V1); });
  LYAP_LAUNCHED("init_store");
}

template <typename T>
void launch_zflush(const void* const* blocks, int nb, int n, int S, const double* Mrows, int t, double* Z,
                   int64_t ldz, int grid, hipStream_t st) {
  if (nb <= 0 || t <= 0) return;
  LYAP_SWITCH_S(S, {
    constexpr int QB = (64 / S) > 0 ? 64 / S : 1;
    int done = 0;
    while (done < nb) {
      const int cnt = nb - done < QB ? nb - done : QB;
      BlockList bl{};
      for (int b = 0; b < cnt; ++b) bl.p[b] = blocks[done + b];
      hipLaunchKernelGGL((k_zflush<T, S>), dim3(grid), dim3(kBlock), 0, st, bl, cnt, n,
                         Mrows + (size_t)done * S * t, t, Z, ldz);
      done += cnt;
    }
  });
  LYAP_LAUNCHED("zflush");
}

int zflush_max_blocks(int S) { return (64 / S) > 0 ? 64 / S : 1; }

template <typename T>
void launch_apply(const OpDev<T>& op, int S, const T* V, T* W, int grid, hipStream_t st) {
  LYAP_SWITCH_S(S, { hipLaunchKernelGGL((k_apply<T, S>), dim3(grid), dim3(kBlock), 0, st, op, V, W); });
  LYAP_LAUNCHED("apply");
}

#define LYAP_INST(T)                                                                                         \
  template void launch_step<T>(const StepArgs<T>&, int, int, hipStream_t);                                  \
  template void launch_replay<T>(const OpDev<T>&, int, const T*, const T*, T*, const double*, int, hipStream_t); \
  template void launch_init<T>(const double*, int64_t, int, int, double*, double*, unsigned*, int*, T*, int,   \
                               hipStream_t);                                                                 \
  template void launch_init_store<T>(const double*, int64_t, int, int, const double*, T*, int, hipStream_t);  \
  template void launch_zflush<T>(const void* const*, int, int, int, const double*, int, double*, int64_t, int, \
                                 hipStream_t);                                                               \
  template void launch_apply<T>(const OpDev<T>&, int, const T*, T*, int, hipStream_t);

LYAP_INST(float)
LYAP_INST(double)

}  // namespace lyap

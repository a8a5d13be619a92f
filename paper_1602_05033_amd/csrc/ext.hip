// lyap_solve over the extended Krylov space EK_m(A, C) (Section 4).
//
// Blocks have ell = 2s columns, [V^(1), V^(2)], stored row-interleaved in FP64.
// One step j:
//   AV  = A V_j                                   (ell columns; kept for T_m)
//   W   = [ (A V_j)^(1), A^{-1} V_j^(2) ]         (inner PCG, FP64)
//   W  -= V (V^T W), twice, against every stored block (block classical
//         Gram-Schmidt with reorthogonalisation; the paper allows the local
//         Lanczos step, which loses orthogonality on these operators)
//   W   = V_{j+1} R by Cholesky-QR twice (positive diagonal)
//   T   : diagonal block sym(V_j^T AV), sub-diagonal block V_{j+1}^T AV
//         (formed directly; the recurrence from H_m is not printed in the
//         paper), written into the (ell+1) x k lower band of T_m
// The residual is Proposition 1 / Algorithm 3 with ell = 2s and the first s
// rows tau-bar of tau_{m+1,m} (its lower s rows vanish, Section 4); Z is
// V_m (Q_m Y-check) from the stored basis.
#include <algorithm>
#include <cmath>
#include <memory>
#include <type_traits>

#include "check.hpp"
#include "lanczos.hpp"
#include "pcg.hpp"
#include "pcnet.hpp"
#include "small.hpp"
#include "solver.hpp"
#include "sylv.hpp"

namespace lyap {

constexpr int kExtThreads = 256;

// Learned inner preconditioner: width, SplitMix64 seed and scale of the
// initial weights, harvest cadence and count, Adam steps and learning rate.
constexpr int kPcC = 2;
constexpr uint64_t kPcSeed = 0x5eedULL;
constexpr double kPcScale = 0.05;
// (50 steps at 1e-2 reach the iteration counts of 200 at 2e-3 on the 100^3
// lognormal operator -- 122 against 119 per solve -- in a quarter of the time)
constexpr int kPcEvery = 16, kPcKeep = 16, kPcSteps = 50;
constexpr double kPcLr = 1e-2;

// C (n x S column-major, leading dimension ldc) -> row-interleaved n x S.
template <int S>
__global__ void k_ext_pack(const double* __restrict__ C, int64_t ldc, int n, double* __restrict__ out) {
  for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < n; r += gridDim.x * blockDim.x) {
    double v[S];
#pragma unroll
    for (int c = 0; c < S; ++c) v[c] = C[(size_t)c * ldc + r];
    store_row<double, S>(out + (size_t)r * S, v);
  }
}

// out (n x S) = columns [S, 2S) of the n x 2S block V.
template <int S>
__global__ void k_ext_split(const double* __restrict__ V, int n, double* __restrict__ out) {
  for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < n; r += gridDim.x * blockDim.x) {
    double v[2 * S], o[S];
    load_row<double, 2 * S>(V + (size_t)r * 2 * S, v);
#pragma unroll
    for (int c = 0; c < S; ++c) o[c] = v[S + c];
    store_row<double, S>(out + (size_t)r * S, o);
  }
}

// W (n x 2S) = [first S columns of A1 (row stride lda1), X (n x S)].
template <int S>
__global__ void k_ext_merge(const double* __restrict__ A1, int lda1, const double* __restrict__ X, int n,
                            double* __restrict__ W) {
  for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < n; r += gridDim.x * blockDim.x) {
    double w[2 * S];
#pragma unroll
    for (int c = 0; c < S; ++c) {
      w[c] = A1[(size_t)r * lda1 + c];
      w[S + c] = X[(size_t)r * S + c];
    }
    store_row<double, 2 * S>(W + (size_t)r * 2 * S, w);
  }
}

// Gram partials of up to NB consecutive blocks against Y in one pass over Y
// (Y is read once per NB blocks instead of once per block):
// part[(b * G + g) * L*L + p*L + q] = sum over the rows of workgroup g of
// X_b[r][p] * Y[r][q], b = blockIdx.y * NB + i < nb; grid (G, ceil(nb / NB)).
template <int L>
constexpr int gram_chunk() {
  return L <= 2 ? 8 : (L <= 4 ? 4 : 1);
}

template <int L>
__global__ __launch_bounds__(kExtThreads) void k_ext_gram(const double* const* X, int nb, const double* __restrict__ Y,
                                                         int n, double* part) {
  constexpr int NB = gram_chunk<L>();
  constexpr int LL = L * L, K = NB * LL;
  __shared__ double red[pow2_at_least(K) * (kExtThreads / 64)];
  const int b0 = blockIdx.y * NB;
  const int nbl = min(NB, nb - b0);  // blocks of this chunk (uniform)
  const double* Xb[NB];
#pragma unroll
  for (int i = 0; i < NB; ++i) Xb[i] = X[b0 + (i < nbl ? i : 0)];
  double acc[K];
#pragma unroll
  for (int e = 0; e < K; ++e) acc[e] = 0.0;
  for (int r = blockIdx.x * kExtThreads + threadIdx.x; r < n; r += gridDim.x * kExtThreads) {
    double y[L], x[NB][L];
    load_row<double, L>(Y + (size_t)r * L, y);
#pragma unroll
    for (int i = 0; i < NB; ++i)
      if (i < nbl) load_row<double, L>(Xb[i] + (size_t)r * L, x[i]);
#pragma unroll
    for (int i = 0; i < NB; ++i)
      if (i < nbl)
#pragma unroll
        for (int p = 0; p < L; ++p)
#pragma unroll
          for (int q = 0; q < L; ++q) acc[i * LL + p * L + q] = fma(x[i][p], y[q], acc[i * LL + p * L + q]);
  }
  block_sum<K, kExtThreads>(acc, red);
  if (threadIdx.x < K) {
    const int i = threadIdx.x / LL, e = threadIdx.x - i * LL;
    if (i < nbl) part[((size_t)(b0 + i) * gridDim.x + blockIdx.x) * LL + e] = red[threadIdx.x];
  }
}

// H[b * LL + e] = sum_g part[(b * G + g) * LL + e]: one wave per entry (lanes
// take g = lane, lane + 64, ..., then a butterfly; a fixed order).
__global__ __launch_bounds__(256) void k_ext_sum(const double* __restrict__ part, int G, int nb, int LL,
                                                 double* __restrict__ H) {
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (i >= nb * LL) return;  // the whole wave
  const int b = i / LL, e = i - b * LL;
  const double* src = part + (size_t)b * G * LL + e;
  double s = 0.0;
  for (int g = lane; g < G; g += 64) s += src[(size_t)g * LL];
  s = wave_sum(s);
  if (lane == 0) H[i] = s;
}

// W -= sum_b X_b H_b; the rows of U blocks are loaded before they are used
// (one 16-byte row per block and thread would leave too few bytes in flight).
template <int L>
__global__ __launch_bounds__(kExtThreads) void k_ext_update(const double* const* X, int nb, const double* __restrict__ H,
                                                           double* __restrict__ W, int n) {
  constexpr int U = L <= 2 ? 8 : (L <= 4 ? 4 : 2);
  constexpr int LL = L * L;
  for (int r = blockIdx.x * kExtThreads + threadIdx.x; r < n; r += gridDim.x * kExtThreads) {
    double acc[L];
#pragma unroll
    for (int c = 0; c < L; ++c) acc[c] = 0.0;
    int b = 0;
    for (; b + U <= nb; b += U) {
      double x[U][L];
#pragma unroll
      for (int u = 0; u < U; ++u) load_row<double, L>(X[b + u] + (size_t)r * L, x[u]);
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const double* h = H + (size_t)(b + u) * LL;
#pragma unroll
        for (int a = 0; a < L; ++a)
#pragma unroll
          for (int c = 0; c < L; ++c) acc[c] = fma(x[u][a], h[a * L + c], acc[c]);
      }
    }
    for (; b < nb; ++b) {
      double x[L];
      load_row<double, L>(X[b] + (size_t)r * L, x);
      const double* h = H + (size_t)b * LL;
#pragma unroll
      for (int a = 0; a < L; ++a)
#pragma unroll
        for (int c = 0; c < L; ++c) acc[c] = fma(x[a], h[a * L + c], acc[c]);
    }
    double w[L];
    load_row<double, L>(W + (size_t)r * L, w);
#pragma unroll
    for (int c = 0; c < L; ++c) w[c] -= acc[c];
    store_row<double, L>(W + (size_t)r * L, w);
  }
}

// Cholesky of the Gram matrix G (L x L): out[0..LL) = R, out[LL..2LL) = R^{-1},
// out[2LL..3LL) = R * Rprev (or R), out[3LL] = trace of the first s diagonal
// entries of G.  flags[0] = tag on a numerically dependent block, flags[1] =
// tag on a non-finite Gram matrix (first occurrence kept).
template <int L>
__global__ void k_ext_chol(const double* G, const double* Rprev, double* out, int s, int* flags, int tag) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  double R[L * L], Ri[L * L], Rt[L * L];
  const double ratio = chol_upper<L>(G, R);
  inv_upper<L>(R, Ri);
  if (Rprev) mul_upper<L>(R, Rprev, Rt);
  else
    for (int i = 0; i < L * L; ++i) Rt[i] = R[i];
  bool finite = true;
  double tr = 0.0;
  for (int i = 0; i < L * L; ++i) {
    finite = finite && isfinite(G[i]) && isfinite(Ri[i]);
    out[i] = R[i];
    out[L * L + i] = Ri[i];
    out[2 * L * L + i] = Rt[i];
  }
  for (int i = 0; i < s; ++i) tr += G[i * L + i];
  out[3 * L * L] = tr;
  if (!(ratio > kBreakdownRatio) && flags[0] == 0) flags[0] = tag;
  if (!finite && flags[1] == 0) flags[1] = tag;
}

// out = W R^{-1} (R^{-1} upper triangular, row-major).
template <int L>
__global__ __launch_bounds__(kExtThreads) void k_ext_scale(const double* W, const double* __restrict__ Ri,
                                                          double* out, int n) {
  for (int r = blockIdx.x * kExtThreads + threadIdx.x; r < n; r += gridDim.x * kExtThreads) {
    double w[L], u[L];
    load_row<double, L>(W + (size_t)r * L, w);
#pragma unroll
    for (int c = 0; c < L; ++c) {
      double acc = 0.0;
#pragma unroll
      for (int a = 0; a <= c; ++a) acc = fma(w[a], Ri[a * L + c], acc);
      u[c] = acc;
    }
    store_row<double, L>(out + (size_t)r * L, u);
  }
}

// Diagonal block j = sym(H0), sub-diagonal block (j+1, j) = H1 into the band
// (band[col * (L+1) + row - col]); H1 is also logged as tau_{j+1,j}.
template <int L>
__global__ void k_ext_tband(const double* H, double* band, int j, double* taulog) {
  const int e = threadIdx.x;
  if (e >= L * L) return;
  const int a = e / L, b = e - a * L;
  const double* H0 = H;
  const double* H1 = H + L * L;
  const size_t ld = L + 1;
  if (a >= b) band[(size_t)(j * L + b) * ld + (a - b)] = 0.5 * (H0[a * L + b] + H0[b * L + a]);
  if (a <= b) band[(size_t)(j * L + b) * ld + (L + a - b)] = H1[a * L + b];
  taulog[(size_t)j * L * L + e] = H1[e];
}

// gamma (L x L, row-major) = first s columns of R, zero elsewhere.
template <int L>
__global__ void k_ext_gamma(const double* R, int s, double* gamma) {
  const int e = threadIdx.x;
  if (e >= L * L) return;
  gamma[e] = (e % L) < s ? R[e] : 0.0;
}

// ------------------------------------------------------------------ host
namespace {

struct ExtWork {
  int n, S, L;
  int G;   // Gram partials per block (workgroups along the rows)
  int Gu;  // workgroups of the row sweeps (update, scale)
  hipStream_t st;
  DevBuf part, H, small, flags;
  size_t part_blocks = 0;
  void ensure(int nb) {
    if ((size_t)nb <= part_blocks) return;
    size_t cap = std::max<size_t>(nb, part_blocks * 2);
    cap = std::max<size_t>(cap, 16);
    LYAP_HIP(hipStreamSynchronize(st));  // the old buffers may still be in use
    part.alloc(cap * G * L * L * sizeof(double));
    H.alloc(cap * L * L * sizeof(double));
    part_blocks = cap;
  }
};

template <int L>
void gram(ExtWork& w, const double* const* X, int nb, const double* Y) {
  constexpr int NB = gram_chunk<L>();
  w.ensure(nb);
  hipLaunchKernelGGL((k_ext_gram<L>), dim3(w.G, (nb + NB - 1) / NB), dim3(kExtThreads), 0, w.st, X, nb, Y, w.n,
                     w.part.as<double>());
  LYAP_LAUNCHED("k_ext_gram");
  const int tot = nb * L * L;
  hipLaunchKernelGGL(k_ext_sum, dim3((tot + 3) / 4), dim3(256), 0, w.st, w.part.as<double>(), w.G, nb, L * L,
                     w.H.as<double>());
  LYAP_LAUNCHED("k_ext_sum");
}

// Cholesky-QR twice: out = W R^{-1}, R = R2 R1 at small + 2LL (slot 'dst').
template <int L>
void cholqr2(ExtWork& w, const double* const* wlist, double* W, const double* const* olist, double* out,
             double* Rdst, int tag) {
  constexpr int LL = L * L;
  double* sm = w.small.as<double>();
  gram<L>(w, wlist, 1, W);
  hipLaunchKernelGGL((k_ext_chol<L>), dim3(1), dim3(64), 0, w.st, w.H.as<double>(), (const double*)nullptr, sm, w.S,
                     w.flags.as<int>(), tag);
  hipLaunchKernelGGL((k_ext_scale<L>), dim3(w.Gu), dim3(kExtThreads), 0, w.st, W, sm + LL, out, w.n);
  gram<L>(w, olist, 1, out);
  hipLaunchKernelGGL((k_ext_chol<L>), dim3(1), dim3(64), 0, w.st, w.H.as<double>(), sm, sm + 4 * LL, w.S,
                     w.flags.as<int>(), tag);
  hipLaunchKernelGGL((k_ext_scale<L>), dim3(w.Gu), dim3(kExtThreads), 0, w.st, out, sm + 5 * LL, out, w.n);
  LYAP_HIP(hipMemcpyAsync(Rdst, sm + 6 * LL, LL * sizeof(double), hipMemcpyDeviceToDevice, w.st));
  LYAP_LAUNCHED("cholqr2");
}

// One extended Krylov space EK_m(A, C) on the device: the operator, its inner
// CG, the stored basis, T_m's band, the tau log and the flags.  lyap_solve
// (method EXT) drives one, sylv_solve (method EXT) two in lockstep.
template <int S>
class ExtSide {
 public:
  static constexpr int L = 2 * S;
  static constexpr int LL = L * L;

  ExtSide(const lyap_op* A, const lyap_opts& o, hipStream_t st, KernelTimer* kt) : st_(st), kt_(kt) {
    n_ = (int)A->n;
    maxit_ = o.max_iter;
    make_op_f64(A, op_, st);
    cg_.reset(new InnerCG(op_.dev, n_, S, o.inner_pc, o.inner_tol, o.inner_max_iter, st));
    blkL_ = (size_t)n_ * L * sizeof(double);
    blkS_ = (size_t)n_ * S * sizeof(double);
    eg_ = grid_for(n_, 1, 1024);
    w_.n = n_;
    w_.S = S;
    w_.L = L;
    w_.G = grid_for(n_, 1, 1024);
    w_.Gu = grid_for(n_, 1, 2048);
    w_.st = st;
    w_.small.alloc(9 * LL * sizeof(double));
    w_.flags.alloc(64);
    LYAP_HIP(hipMemsetAsync(w_.flags.p, 0, 64, st));
    V_.reserve((size_t)maxit_ + 2);
    ptrs_.alloc(((size_t)maxit_ + 2) * sizeof(void*));
    hptrs_.alloc(((size_t)maxit_ + 2) * sizeof(void*));
    wlist_.alloc(sizeof(void*));
    AV_.alloc(blkL_);
    W_.alloc(blkL_);
    Bs_.alloc(blkS_);
    Xs_.alloc(blkS_);
    band_.alloc((size_t)(L + 1) * L * (maxit_ + 2) * sizeof(double));
    taulog_.alloc(((size_t)maxit_ + 1) * LL * sizeof(double));
    R0_.alloc(LL * sizeof(double));
    gamma_.alloc(LL * sizeof(double));
    LYAP_HIP(hipMemsetAsync(band_.p, 0, band_.bytes, st));
    const void* wp = W_.p;
    LYAP_HIP(hipMemcpy(wlist_.p, &wp, sizeof(void*), hipMemcpyHostToDevice));
  }

  InnerCG& cg() { return *cg_; }
  const OpHolder<double>& op() const { return op_; }
  int n() const { return n_; }
  int m() const { return m_; }
  double beta() const { return beta_; }
  const double* band() const { return band_.as<double>(); }
  const double* gamma() const { return gamma_.as<double>(); }
  const double* tau(int mm) const { return taulog_.as<double>() + (size_t)(mm - 1) * LL; }
  const void* block(int i) const { return V_[i].p; }

  void read_flags(int* f) {
    LYAP_HIP(hipMemcpyAsync(f, w_.flags.p, 2 * sizeof(int), hipMemcpyDeviceToHost, st_));
    LYAP_HIP(hipStreamSynchronize(st_));
  }

  // Start, first half: B = C packed, X = A^{-1} C (the inner solve).
  void start_solve(const double* C, int64_t ldc) {
    hipLaunchKernelGGL((k_ext_pack<S>), dim3(eg_), dim3(kBlock), 0, st_, C, ldc, n_, Bs_.as<double>());
    cg_->solve(Bs_.as<double>(), Xs_.as<double>(), kt_);
  }

  // Start, second half: [C, A^{-1} C] = V_1 R, gamma = R[:, :s]; beta = ||C||_F.
  void start_finish() {
    hipLaunchKernelGGL((k_ext_merge<S>), dim3(eg_), dim3(kBlock), 0, st_, Bs_.as<double>(), S, Xs_.as<double>(), n_,
                       W_.as<double>());
    LYAP_LAUNCHED("ext start");
    double* V1 = new_block();
    if (kt_) kt_->mark(LYAP_K_INIT);
    cholqr2<L>(w_, dwl(), W_.as<double>(), dptrs(), V1, R0_.as<double>(), -1);
    hipLaunchKernelGGL((k_ext_gamma<L>), dim3(1), dim3(64), 0, st_, R0_.as<double>(), S, gamma_.as<double>());
    if (kt_) kt_->collect();
    int f[2];
    std::vector<double> g(LL);
    LYAP_HIP(hipMemcpyAsync(g.data(), gamma_.p, LL * sizeof(double), hipMemcpyDeviceToHost, st_));
    read_flags(f);
    double tr = 0.0;
    bool fin = true;
    for (double v : g) {
      tr += v * v;
      fin = fin && std::isfinite(v);
    }
    LYAP_REQUIRE(f[1] == 0 && fin, LYAP_E_NUMERIC, "C contains NaN or Inf");
    LYAP_REQUIRE(tr > 0.0, LYAP_E_ARG, "C is zero");
    LYAP_REQUIRE(f[0] == 0, LYAP_E_BREAKDOWN,
                 "[C, A^{-1} C] is numerically rank deficient (deflation not implemented)");
    beta_ = std::sqrt(tr);  // ||C||_F = ||gamma||_F
  }

  // One step: V_{m+1} and T_m's block column m.
  void step() {
    const int j = m_;
    // the next block is allocated first, while the device still works on the
    // previous step (the inner solve ends with a host wait)
    double* Vn = new_block();
    const double* Vj = V_[j].as<double>();
    launch_apply<double>(op_.dev, L, Vj, AV_.as<double>(), eg_, st_);
    hipLaunchKernelGGL((k_ext_split<S>), dim3(eg_), dim3(kBlock), 0, st_, Vj, n_, Bs_.as<double>());
    cg_->solve(Bs_.as<double>(), Xs_.as<double>(), kt_);
    if (kt_) kt_->mark(LYAP_K_EXT_ORTH);
    hipLaunchKernelGGL((k_ext_merge<S>), dim3(eg_), dim3(kBlock), 0, st_, AV_.as<double>(), L, Xs_.as<double>(), n_,
                       W_.as<double>());
    for (int sweep = 0; sweep < 2; ++sweep) {
      gram<L>(w_, dptrs(), j + 1, W_.as<double>());
      hipLaunchKernelGGL((k_ext_update<L>), dim3(w_.Gu), dim3(kExtThreads), 0, st_, dptrs(), j + 1,
                         w_.H.as<double>(), W_.as<double>(), n_);
      LYAP_LAUNCHED("k_ext_update");
    }
    cholqr2<L>(w_, dwl(), W_.as<double>(), dptrs() + j + 1, Vn, w_.small.as<double>() + 8 * LL, j + 1);
    gram<L>(w_, dptrs() + j, 2, AV_.as<double>());
    hipLaunchKernelGGL((k_ext_tband<L>), dim3(1), dim3(64), 0, st_, w_.H.as<double>(), band_.as<double>(), j,
                       taulog_.as<double>());
    LYAP_LAUNCHED("k_ext_tband");
    ++m_;
  }

  // Host copies of T_m's band (ld = L + 1, entries past k cleared) and of tau.
  double* band_host(int mm) const {
    const int k = mm * L;
    double* h = (double*)std::malloc((size_t)(L + 1) * k * sizeof(double));
    LYAP_HIP(hipMemcpy(h, band_.p, (size_t)(L + 1) * k * sizeof(double), hipMemcpyDeviceToHost));
    for (int c = 0; c < k; ++c)
      for (int d = 0; d <= L; ++d)
        if (c + d >= k) h[(size_t)c * (L + 1) + d] = 0.0;
    return h;
  }

 private:
  // A new basis block; its address goes to the device table from a pinned
  // slot written once (an ordered asynchronous copy, no host wait).
  double* new_block() {
    V_.emplace_back(blkL_);
    const size_t i = V_.size() - 1;
    hptrs_.as<const void*>()[i] = V_.back().p;
    LYAP_HIP(hipMemcpyAsync(ptrs_.as<const void*>() + i, hptrs_.as<const void*>() + i, sizeof(void*),
                            hipMemcpyHostToDevice, st_));
    return V_.back().as<double>();
  }
  const double* const* dptrs() const { return ptrs_.as<const double*>(); }
  const double* const* dwl() const { return wlist_.as<const double*>(); }

  hipStream_t st_;
  KernelTimer* kt_;
  int n_ = 0, maxit_ = 0, m_ = 0, eg_ = 1;
  size_t blkL_ = 0, blkS_ = 0;
  double beta_ = 0.0;
  OpHolder<double> op_;
  std::unique_ptr<InnerCG> cg_;
  ExtWork w_;
  std::vector<DevBuf> V_;
  DevBuf ptrs_, wlist_, AV_, W_, Bs_, Xs_, band_, taulog_, R0_, gamma_;
  HostBuf hptrs_;
};

template <int S>
lyap_status ext_impl(const lyap_op* A, const double* C, int64_t ldc, const lyap_opts& o, lyap_result* out) {
  constexpr int L = 2 * S;
  constexpr int LL = L * L;
  const auto t_entry = Clock::now();
  hipStream_t st = (hipStream_t)o.stream;
  const int n = (int)A->n;
  out->n = n;
  out->s = S;
  out->ell = L;
  KernelTimer kt;
  kt.st = st;
  kt.on = o.profile != 0;
  const int maxit = o.max_iter;
  ExtSide<S> side(A, o, st, &kt);
  InnerCG& cg = side.cg();
  DevBuf chk(sizeof(CheckOut));
  HostBuf hchk(sizeof(CheckOut));

  // ---- start: [C, A^{-1} C] = V_1 R, gamma = R[:, :s]
  const auto t_pass1 = Clock::now();
  std::unique_ptr<PcNetGpu> net;
  double train_ms = 0.0;
  if (o.inner_pc == LYAP_PC_LEARNED) {
    net = cg.make_schur_net(kPcC);
    std::vector<float> W(pcnet_param_count(kPcC));
    pcnet_init_weights(kPcC, kPcSeed, kPcScale, W.data());
    net->set_weights(W.data());
    cg.harvest(kPcEvery, kPcKeep);
  }
  side.start_solve(C, ldc);
  if (net) {
    // train on the start solve's own iterates, then switch to flexible CG
    const auto t_tr = Clock::now();
    std::vector<int> use;
    std::vector<double> eAe;
    for (int i = 0; i < cg.pairs(); ++i) {
      const double v = net->energy(cg.pair_e(i));
      if (v > 0.0) {
        use.push_back(i);
        eAe.push_back(v);
      }
    }
    LYAP_REQUIRE(!use.empty(), LYAP_E_INNER, "no training pairs from the first inner solve");
    for (int t = 0; t < kPcSteps; ++t) {
      const int q = t % (int)use.size();
      net->grad(cg.pair_r(use[q]), cg.pair_e(use[q]), eAe[q], false);
      net->adam(kPcLr);
    }
    LYAP_HIP(hipStreamSynchronize(st));
    train_ms = ms_since(t_tr);
    cg.set_net_schur(net.get());
  }
  side.start_finish();
  out->beta = side.beta();
  const double beta2 = out->beta * out->beta;

  Checker ck(L, S, st);
  CheckSchedule sched{o.check_every, maxit};
  std::vector<int> hm;
  std::vector<double> hr;
  double check_ms = 0.0, t_to_tol = 0.0, lam_absmax = 0.0, last_res = INFINITY;
  int next_check = sched.first();
  int m = 0, checked_m = 0;
  lyap_status status = LYAP_NOT_CONVERGED;

  auto run_check = [&](int mm) {
    const auto t0 = Clock::now();
    kt.mark(LYAP_K_CHECK);
    ck.run(side.band(), mm * L, side.gamma(), side.tau(mm), chk.as<CheckOut>());
    kt.collect();
    LYAP_HIP(hipMemcpyAsync(hchk.p, chk.p, sizeof(CheckOut), hipMemcpyDeviceToHost, st));
    LYAP_HIP(hipStreamSynchronize(st));
    check_ms += ms_since(t0);
    checked_m = mm;
    const CheckOut& c = *hchk.as<CheckOut>();
    lam_absmax = std::max(std::fabs(c.lam_min), std::fabs(c.lam_max));
    out->n_checks++;
    return c;
  };

  while (m < maxit) {
    side.step();
    ++m;
    if (m == next_check || m == maxit) {
      int f[2];
      side.read_flags(f);
      LYAP_REQUIRE(f[1] == 0, LYAP_E_NUMERIC, "non-finite values in the extended Krylov basis at step %d", f[1]);
      int mm = m;
      const bool broke = f[0] > 0 && f[0] <= m;
      if (broke) mm = f[0];  // the QR at step f[0]-1 found a dependent block
      CheckOut c = run_check(mm);
      LYAP_REQUIRE(std::isfinite(c.res), LYAP_E_NUMERIC, "residual is not finite at m=%d", mm);
      const double rel = c.res / beta2;
      hm.push_back(mm);
      hr.push_back(rel);
      last_res = rel;
      if (o.verbose) std::fprintf(stderr, "[lyap-ext] m=%d k=%d res=%.3e\n", mm, mm * L, rel);
      LYAP_REQUIRE(c.lam_max < 0.0, LYAP_E_INDEFINITE,
                   "Ritz value %.3e >= 0 at m=%d: the operator is not negative definite", c.lam_max, mm);
      if (rel <= o.tol) {
        status = LYAP_OK;
        m = mm;
        t_to_tol = ms_since(t_entry);
        break;
      }
      if (broke) {
        m = mm;
        status = LYAP_E_BREAKDOWN;
        set_error("extended Krylov breakdown at m=%d with residual %.3e above tol", mm, rel);
        break;
      }
      next_check = sched.next(m, rel, o.tol);
    }
  }
  if (checked_m != m) {
    CheckOut c = run_check(m);
    hm.push_back(m);
    hr.push_back(c.res / beta2);
    last_res = c.res / beta2;
  }
  const double pass1_ms = ms_since(t_pass1) - check_ms;
  out->m = m;
  out->res = last_res;
  store_history(out, hm, hr);

  // ---- finalisation
  const auto t_fin = Clock::now();
  std::vector<double> tau_h(LL);
  LYAP_HIP(hipMemcpyAsync(tau_h.data(), side.tau(m), LL * sizeof(double), hipMemcpyDeviceToHost, st));
  LYAP_HIP(hipStreamSynchronize(st));
  double tau_f = 0.0;
  for (double v : tau_h) tau_f += v * v;
  tau_f = std::sqrt(tau_f);
  double eps = o.trunc_eps;
  if (!(eps >= 0.0)) eps = std::min(1e-12, 0.05 * o.tol / (lam_absmax + tau_f)) * beta2;
  out->trunc_eps = eps;
  DevBuf M;
  kt.mark(LYAP_K_FINAL);
  const int t = finalise_factor(ck, side.band(), side.gamma(), eps, M, st);
  kt.collect();
  out->t = t;
  const double fin_ms = ms_since(t_fin);

  // ---- Z = V_m M from the stored basis
  const auto t_z = Clock::now();
  bool owned = false;
  out->Z = alloc_output(o, (size_t)n * std::max(t, 1) * sizeof(double), &owned);
  out->owns_Z = owned ? 1 : 0;
  if (t > 0) {
    LYAP_HIP(hipMemsetAsync(out->Z, 0, (size_t)n * t * sizeof(double), st));
    std::vector<const void*> bp;
    for (int i = 0; i < m; ++i) bp.push_back(side.block(i));
    kt.mark(LYAP_K_ZFLUSH);
    launch_zflush<double>(bp.data(), m, n, L, M.as<double>(), t, out->Z, n, 0, st);
  }
  LYAP_HIP(hipStreamSynchronize(st));
  kt.collect();
  const double z_ms = ms_since(t_z);

  if (o.want_T) {
    out->T_band = side.band_host(m);
    std::vector<double> g(LL);
    LYAP_HIP(hipMemcpy(g.data(), side.gamma(), LL * sizeof(double), hipMemcpyDeviceToHost));
    out->gamma = (double*)std::malloc(LL * sizeof(double));
    out->tau = (double*)std::malloc(LL * sizeof(double));
    for (int a = 0; a < L; ++a)
      for (int b = 0; b < L; ++b) {
        out->gamma[a + b * L] = g[a * L + b];
        out->tau[a + b * L] = tau_h[a * L + b];
      }
  }
  const CgStats& cs = cg.stats();
  out->inner_iters = cs.iters;
  out->n_inner = cs.solves;
  out->times_ms[LYAP_T_PASS1] = pass1_ms;
  out->times_ms[LYAP_T_INNER] = cs.ms;
  out->times_ms[LYAP_T_TRAIN] = train_ms;
  out->times_ms[LYAP_T_CHECKS] = check_ms;
  out->times_ms[LYAP_T_FINAL] = fin_ms;
  out->times_ms[LYAP_T_PASS2] = z_ms;
  out->times_ms[LYAP_T_TOTAL] = ms_since(t_entry);
  out->times_ms[LYAP_T_TO_TOL] = t_to_tol;
  for (int i = 0; i < LYAP_K_COUNT; ++i) {
    out->kern_ms[i] = kt.ms[i];
    out->kern_n[i] = kt.n[i];
  }
  {
    // one iteration kernel of the inner CG (Jacobi: the single-reduction iteration on the
    // whole grid; IC(0): the condensed iteration on the black cells)
    out->kern_bytes[LYAP_K_CG_DIR] = cg.iter_bytes();
    out->kern_bytes[LYAP_K_CG_UPD] = cg.upd_bytes();
    // on the Schur complement the x, r update runs inside the network's first
    // convolution (x, r, p, q in; x, r out at the black slots)
    if (net) out->kern_bytes[LYAP_K_PCNET] = net->apply_bytes() + cg.upd_bytes();
  }
  out->status = status;
  return status;
}

// sylv_solve over EK_m(A, C1) and EK_m(B, C2) (Section 5.1 with the spaces of
// Section 4): the two spaces advance in lockstep, the residual is the
// corrected Algorithm 4 with ell = 2s and the first s rows of tau_{m+1,m} and
// iota_{m+1,m}, and the truncated factors come from the stored bases.
template <int S>
lyap_status sylv_ext_impl(const lyap_op* A, const lyap_op* B, const double* C1, int64_t ldc1, const double* C2,
                          int64_t ldc2, const lyap_opts& o, sylv_result* out) {
  constexpr int L = 2 * S;
  constexpr int LL = L * L;
  const auto t_entry = Clock::now();
  hipStream_t st = (hipStream_t)o.stream;
  const int n1 = (int)A->n, n2 = (int)B->n;
  out->n1 = n1;
  out->n2 = n2;
  out->s = S;
  out->ell = L;
  const int maxit = o.max_iter;
  KernelTimer kt;
  kt.st = st;
  kt.on = o.profile != 0;
  ExtSide<S> sa(A, o, st, &kt), sb(B, o, st, &kt);
  const auto t_pass1 = Clock::now();
  sa.start_solve(C1, ldc1);
  sa.start_finish();
  sb.start_solve(C2, ldc2);
  sb.start_finish();
  out->beta1 = sa.beta();
  out->beta2 = sb.beta();
  const double b12 = sa.beta() * sb.beta();

  Checker ca(L, S, st), cb(L, S, st);
  DevBuf part(4096 * sizeof(double)), counter(64), chk(sizeof(CheckOut));
  HostBuf hchk(sizeof(CheckOut) + 4 * sizeof(double));
  LYAP_HIP(hipMemsetAsync(counter.p, 0, 64, st));
  CheckSchedule sched{o.check_every, maxit};
  std::vector<int> hm;
  std::vector<double> hr;
  double check_ms = 0.0, t_to_tol = 0.0, lamA_abs = 0.0, lamB_abs = 0.0, last_res = INFINITY;
  int next_check = sched.first(), m = 0, checked_m = 0;
  lyap_status status = LYAP_NOT_CONVERGED;
  CheckOut* hc = hchk.as<CheckOut>();
  double* hl = reinterpret_cast<double*>(hchk.as<char>() + sizeof(CheckOut));

  auto run_check = [&](int mm) -> double {
    const auto t0 = Clock::now();
    kt.mark(LYAP_K_CHECK);
    const int k = mm * L;
    ca.prepare(sa.band(), k, sa.gamma(), sa.tau(mm));
    cb.prepare(sb.band(), k, sb.gamma(), sb.tau(mm));
    launch_sylv_sum(ca, cb, k, L, S, part.as<double>(), counter.as<unsigned>(), chk.as<CheckOut>(), st);
    kt.collect();
    LYAP_HIP(hipMemcpyAsync(hc, chk.p, sizeof(CheckOut), hipMemcpyDeviceToHost, st));
    LYAP_HIP(hipMemcpyAsync(&hl[0], ca.lam(), sizeof(double), hipMemcpyDeviceToHost, st));
    LYAP_HIP(hipMemcpyAsync(&hl[1], ca.lam() + k - 1, sizeof(double), hipMemcpyDeviceToHost, st));
    LYAP_HIP(hipMemcpyAsync(&hl[2], cb.lam(), sizeof(double), hipMemcpyDeviceToHost, st));
    LYAP_HIP(hipMemcpyAsync(&hl[3], cb.lam() + k - 1, sizeof(double), hipMemcpyDeviceToHost, st));
    LYAP_HIP(hipStreamSynchronize(st));
    check_ms += ms_since(t0);
    checked_m = mm;
    out->n_checks++;
    LYAP_REQUIRE(std::isfinite(hc->res), LYAP_E_NUMERIC, "residual is not finite at m=%d", mm);
    const double rel = hc->res / b12;
    hm.push_back(mm);
    hr.push_back(rel);
    last_res = rel;
    lamA_abs = std::max(std::fabs(hl[0]), std::fabs(hl[1]));
    lamB_abs = std::max(std::fabs(hl[2]), std::fabs(hl[3]));
    if (o.verbose) std::fprintf(stderr, "[sylv-ext] m=%d k=%d res=%.3e\n", mm, k, rel);
    LYAP_REQUIRE(hc->lam_max < 0.0, LYAP_E_INDEFINITE,
                 "Ritz value %.3e >= 0 at m=%d: an operator is not negative definite", hc->lam_max, mm);
    return rel;
  };

  while (m < maxit) {
    sa.step();
    sb.step();
    ++m;
    if (m == next_check || m == maxit) {
      int fa[2], fb[2];
      sa.read_flags(fa);
      sb.read_flags(fb);
      LYAP_REQUIRE(fa[1] == 0 && fb[1] == 0, LYAP_E_NUMERIC,
                   "non-finite values in an extended Krylov basis at step %d", std::max(fa[1], fb[1]));
      int bk = 0;
      for (int f : {fa[0], fb[0]})
        if (f > 0 && f <= m && (bk == 0 || f < bk)) bk = f;
      const int mm = bk > 0 ? bk : m;  // the QR at step bk-1 found a dependent block
      const double rel = run_check(mm);
      if (rel <= o.tol) {
        status = LYAP_OK;
        m = mm;
        t_to_tol = ms_since(t_entry);
        break;
      }
      if (bk > 0) {
        m = mm;
        status = LYAP_E_BREAKDOWN;
        set_error("extended Krylov breakdown at m=%d with residual %.3e above tol", mm, rel);
        break;
      }
      next_check = sched.next(m, rel, o.tol);
    }
  }
  if (checked_m != m) run_check(m);
  const double pass1_ms = ms_since(t_pass1) - check_ms;
  out->m = m;
  out->res = last_res;
  out->n_hist = (int)hm.size();
  out->hist_m = (int32_t*)std::malloc(std::max<size_t>(1, hm.size()) * sizeof(int32_t));
  out->hist_res = (double*)std::malloc(std::max<size_t>(1, hr.size()) * sizeof(double));
  for (size_t i = 0; i < hm.size(); ++i) {
    out->hist_m[i] = hm[i];
    out->hist_res[i] = hr[i];
  }

  // ---- finalisation
  const auto t_fin = Clock::now();
  std::vector<double> tau_h(LL), iota_h(LL);
  LYAP_HIP(hipMemcpyAsync(tau_h.data(), sa.tau(m), LL * sizeof(double), hipMemcpyDeviceToHost, st));
  LYAP_HIP(hipMemcpyAsync(iota_h.data(), sb.tau(m), LL * sizeof(double), hipMemcpyDeviceToHost, st));
  LYAP_HIP(hipStreamSynchronize(st));
  auto fro = [](const std::vector<double>& v) {
    double a = 0.0;
    for (double x : v) a += x * x;
    return std::sqrt(a);
  };
  // ||R(Y) - R(Y + dY)|| <= (||T_m underline|| + ||J_m underline||) ||dY||_F
  const double nu = lamA_abs + fro(tau_h) + lamB_abs + fro(iota_h);
  double eps = o.trunc_eps;
  if (!(eps >= 0.0)) eps = std::min(1e-12, 0.05 * o.tol / nu) * b12;
  out->trunc_eps = eps;
  DevBuf M1, M2;
  kt.mark(LYAP_K_FINAL);
  const int t = finalise_sylv(ca, cb, sa.band(), sb.band(), sa.gamma(), sb.gamma(), L, eps, M1, M2, st);
  kt.collect();
  out->t = t;
  const double fin_ms = ms_since(t_fin);

  // ---- Z1 = V_m M1, Z2 = U_m M2 from the stored bases
  const auto t_z = Clock::now();
  bool own1 = false, own2 = false;
  out->Z1 = alloc_output(o, (size_t)n1 * std::max(t, 1) * sizeof(double), &own1);
  out->Z2 = alloc_output(o, (size_t)n2 * std::max(t, 1) * sizeof(double), &own2);
  out->owns_Z = own1 ? 1 : 0;
  if (t > 0) {
    LYAP_HIP(hipMemsetAsync(out->Z1, 0, (size_t)n1 * t * sizeof(double), st));
    LYAP_HIP(hipMemsetAsync(out->Z2, 0, (size_t)n2 * t * sizeof(double), st));
    std::vector<const void*> ba, bb;
    for (int i = 0; i < m; ++i) {
      ba.push_back(sa.block(i));
      bb.push_back(sb.block(i));
    }
    kt.mark(LYAP_K_ZFLUSH);
    launch_zflush<double>(ba.data(), m, n1, L, M1.as<double>(), t, out->Z1, n1, 0, st);
    launch_zflush<double>(bb.data(), m, n2, L, M2.as<double>(), t, out->Z2, n2, 0, st);
  }
  LYAP_HIP(hipStreamSynchronize(st));
  kt.collect();
  const double z_ms = ms_since(t_z);

  if (o.want_T) {
    out->T_band = sa.band_host(m);
    out->J_band = sb.band_host(m);
    auto sq = [&](const double* dev) {
      std::vector<double> g(LL);
      LYAP_HIP(hipMemcpy(g.data(), dev, LL * sizeof(double), hipMemcpyDeviceToHost));
      double* h = (double*)std::malloc(LL * sizeof(double));
      rowmajor_to_colmajor(g.data(), L, L, h);
      return h;
    };
    out->gamma1 = sq(sa.gamma());
    out->gamma2 = sq(sb.gamma());
    out->tau = (double*)std::malloc(LL * sizeof(double));
    out->iota = (double*)std::malloc(LL * sizeof(double));
    rowmajor_to_colmajor(tau_h.data(), L, L, out->tau);
    rowmajor_to_colmajor(iota_h.data(), L, L, out->iota);
  }
  out->times_ms[LYAP_T_PASS1] = pass1_ms;
  out->times_ms[LYAP_T_CHECKS] = check_ms;
  out->times_ms[LYAP_T_FINAL] = fin_ms;
  out->times_ms[LYAP_T_PASS2] = z_ms;
  out->times_ms[LYAP_T_INNER] = sa.cg().stats().ms + sb.cg().stats().ms;
  out->times_ms[LYAP_T_TOTAL] = ms_since(t_entry);
  out->times_ms[LYAP_T_TO_TOL] = t_to_tol;
  for (int i = 0; i < LYAP_K_COUNT; ++i) {
    out->kern_ms[i] = kt.ms[i];
    out->kern_n[i] = kt.n[i];
  }
  out->status = status;
  return status;
}

}  // namespace

template <typename T>
lyap_status solve_ext(const lyap_op* A, const double* C, int S, int64_t ldc, const lyap_opts& o, lyap_result* out) {
  LYAP_REQUIRE((std::is_same_v<T, double>), LYAP_E_UNSUPPORTED,
               "the extended Krylov method runs with FP64 storage only");
  switch (S) {
    case 1: return ext_impl<1>(A, C, ldc, o, out);
    case 2: return ext_impl<2>(A, C, ldc, o, out);
    case 4: return ext_impl<4>(A, C, ldc, o, out);
    default: LYAP_REQUIRE(false, LYAP_E_UNSUPPORTED, "extended Krylov supports s = 1, 2 or 4 (got %d)", S);
  }
  return LYAP_E_UNSUPPORTED;
}

template lyap_status solve_ext<float>(const lyap_op*, const double*, int, int64_t, const lyap_opts&, lyap_result*);
template lyap_status solve_ext<double>(const lyap_op*, const double*, int, int64_t, const lyap_opts&, lyap_result*);

lyap_status solve_sylv_ext(const lyap_op* A, const lyap_op* B, const double* C1, int64_t ldc1, const double* C2,
                           int64_t ldc2, int S, const lyap_opts& o, sylv_result* out) {
  LYAP_REQUIRE(o.storage == LYAP_STORE_F64, LYAP_E_UNSUPPORTED, "the extended Krylov method runs with FP64 storage only");
  LYAP_REQUIRE(o.inner_pc == LYAP_PC_NONE || o.inner_pc == LYAP_PC_JACOBI || o.inner_pc == LYAP_PC_IC0,
               LYAP_E_UNSUPPORTED, "extended Krylov Sylvester solves take inner_pc NONE, JACOBI or IC0");
  switch (S) {
    case 1: return sylv_ext_impl<1>(A, B, C1, ldc1, C2, ldc2, o, out);
    case 2: return sylv_ext_impl<2>(A, B, C1, ldc1, C2, ldc2, o, out);
    case 4: return sylv_ext_impl<4>(A, B, C1, ldc1, C2, ldc2, o, out);
    default: LYAP_REQUIRE(false, LYAP_E_UNSUPPORTED, "extended Krylov supports s = 1, 2 or 4 (got %d)", S);
  }
  return LYAP_E_UNSUPPORTED;
}

}  // namespace lyap

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

namespace lyap {

constexpr int kExtThreads = 256;

// Learned inner preconditioner: width, SplitMix64 seed and scale of the
// initial weights, harvest cadence and count, Adam steps and learning rate.
constexpr int kPcC = 4;
constexpr uint64_t kPcSeed = 0x5eedULL;
constexpr double kPcScale = 0.05;
constexpr int kPcEvery = 32, kPcKeep = 16, kPcSteps = 200;
constexpr double kPcLr = 2e-3;

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

// part[(b * G + g) * L*L + p*L + q] = sum over the rows of workgroup g of
// X_b[r][p] * Y[r][q]; grid (G, nb).
template <int L>
__global__ __launch_bounds__(kExtThreads) void k_ext_gram(const double* const* X, const double* __restrict__ Y, int n,
                                                         double* part) {
  __shared__ double red[pow2_at_least(L * L) * (kExtThreads / 64)];
  const double* __restrict__ Xb = X[blockIdx.y];
  double acc[L * L];
#pragma unroll
  for (int e = 0; e < L * L; ++e) acc[e] = 0.0;
  for (int r = blockIdx.x * kExtThreads + threadIdx.x; r < n; r += gridDim.x * kExtThreads) {
    double x[L], y[L];
    load_row<double, L>(Xb + (size_t)r * L, x);
    load_row<double, L>(Y + (size_t)r * L, y);
#pragma unroll
    for (int p = 0; p < L; ++p)
#pragma unroll
      for (int q = 0; q < L; ++q) acc[p * L + q] = fma(x[p], y[q], acc[p * L + q]);
  }
  write_partial<L * L, kExtThreads>(acc, red, part + (size_t)blockIdx.y * gridDim.x * L * L);
}

// H[b * LL + e] = sum_g part[(b * G + g) * LL + e], in order of g.
__global__ void k_ext_sum(const double* __restrict__ part, int G, int nb, int LL, double* __restrict__ H) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nb * LL) return;
  const int b = i / LL, e = i - b * LL;
  double s = 0.0;
  for (int g = 0; g < G; ++g) s += part[((size_t)b * G + g) * LL + e];
  H[i] = s;
}

// W -= sum_b X_b H_b.
template <int L>
__global__ __launch_bounds__(kExtThreads) void k_ext_update(const double* const* X, int nb, const double* __restrict__ H,
                                                           double* __restrict__ W, int n) {
  for (int r = blockIdx.x * kExtThreads + threadIdx.x; r < n; r += gridDim.x * kExtThreads) {
    double w[L];
    load_row<double, L>(W + (size_t)r * L, w);
    double acc[L];
#pragma unroll
    for (int c = 0; c < L; ++c) acc[c] = 0.0;
    for (int b = 0; b < nb; ++b) {
      double x[L];
      load_row<double, L>(X[b] + (size_t)r * L, x);
      const double* h = H + (size_t)b * L * L;
#pragma unroll
      for (int a = 0; a < L; ++a)
#pragma unroll
        for (int c = 0; c < L; ++c) acc[c] = fma(x[a], h[a * L + c], acc[c]);
    }
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
  int n, S, L, G;
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
  w.ensure(nb);
  hipLaunchKernelGGL((k_ext_gram<L>), dim3(w.G, nb), dim3(kExtThreads), 0, w.st, X, Y, w.n, w.part.as<double>());
  LYAP_LAUNCHED("k_ext_gram");
  const int tot = nb * L * L;
  hipLaunchKernelGGL(k_ext_sum, dim3((tot + 255) / 256), dim3(256), 0, w.st, w.part.as<double>(), w.G, nb, L * L,
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
  hipLaunchKernelGGL((k_ext_scale<L>), dim3(w.G), dim3(kExtThreads), 0, w.st, W, sm + LL, out, w.n);
  gram<L>(w, olist, 1, out);
  hipLaunchKernelGGL((k_ext_chol<L>), dim3(1), dim3(64), 0, w.st, w.H.as<double>(), sm, sm + 4 * LL, w.S,
                     w.flags.as<int>(), tag);
  hipLaunchKernelGGL((k_ext_scale<L>), dim3(w.G), dim3(kExtThreads), 0, w.st, out, sm + 5 * LL, out, w.n);
  LYAP_HIP(hipMemcpyAsync(Rdst, sm + 6 * LL, LL * sizeof(double), hipMemcpyDeviceToDevice, w.st));
  LYAP_LAUNCHED("cholqr2");
}

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
  OpHolder<double> op;
  make_op_f64(A, op, st);
  InnerCG cg(op.dev, n, S, o.inner_pc, o.inner_tol, o.inner_max_iter, st);
  KernelTimer kt;
  kt.st = st;
  kt.on = o.profile != 0;

  const int maxit = o.max_iter;
  const size_t blkL = (size_t)n * L * sizeof(double);
  const size_t blkS = (size_t)n * S * sizeof(double);
  const int eg = grid_for(n, 1, 1024);

  ExtWork w;
  w.n = n;
  w.S = S;
  w.L = L;
  w.G = stream_grid(n);
  w.st = st;
  w.small.alloc(9 * LL * sizeof(double));
  w.flags.alloc(64);
  LYAP_HIP(hipMemsetAsync(w.flags.p, 0, 64, st));

  std::vector<DevBuf> V;
  V.reserve((size_t)maxit + 2);
  DevBuf ptrs(((size_t)maxit + 2) * sizeof(void*));
  DevBuf wlist(sizeof(void*));
  DevBuf AV(blkL), W(blkL), Bs(blkS), Xs(blkS);
  DevBuf band((size_t)(L + 1) * L * (maxit + 2) * sizeof(double));
  DevBuf taulog(((size_t)maxit + 1) * LL * sizeof(double));
  DevBuf R0(LL * sizeof(double)), gamma(LL * sizeof(double));
  DevBuf chk(sizeof(CheckOut));
  HostBuf hchk(sizeof(CheckOut));
  LYAP_HIP(hipMemsetAsync(band.p, 0, band.bytes, st));
  {
    const void* wp = W.p;
    LYAP_HIP(hipMemcpy(wlist.p, &wp, sizeof(void*), hipMemcpyHostToDevice));
  }
  const double* const* dptrs = ptrs.as<const double*>();
  const double* const* dwl = wlist.as<const double*>();
  auto new_block = [&]() {
    V.emplace_back(blkL);
    const void* p = V.back().p;
    LYAP_HIP(hipMemcpy(ptrs.as<const void*>() + (V.size() - 1), &p, sizeof(void*), hipMemcpyHostToDevice));
    return V.back().as<double>();
  };
  auto read_flags = [&](int* f) {
    LYAP_HIP(hipMemcpyAsync(f, w.flags.p, 2 * sizeof(int), hipMemcpyDeviceToHost, st));
    LYAP_HIP(hipStreamSynchronize(st));
  };

  // ---- start: [C, A^{-1} C] = V_1 R, gamma = R[:, :s]
  const auto t_pass1 = Clock::now();
  hipLaunchKernelGGL((k_ext_pack<S>), dim3(eg), dim3(kBlock), 0, st, C, ldc, n, Bs.as<double>());
  std::unique_ptr<PcNetGpu> net;
  double train_ms = 0.0;
  if (o.inner_pc == LYAP_PC_LEARNED) {
    net = std::make_unique<PcNetGpu>(op.dev, kPcC, st);
    std::vector<float> W(pcnet_param_count(kPcC));
    pcnet_init_weights(kPcC, kPcSeed, kPcScale, W.data());
    net->set_weights(W.data());
    cg.harvest(kPcEvery, kPcKeep);
  }
  cg.solve(Bs.as<double>(), Xs.as<double>(), &kt);
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
    cg.set_net(net.get());
  }
  hipLaunchKernelGGL((k_ext_merge<S>), dim3(eg), dim3(kBlock), 0, st, Bs.as<double>(), S, Xs.as<double>(), n,
                     W.as<double>());
  LYAP_LAUNCHED("ext start");
  double* V1 = new_block();
  kt.mark(LYAP_K_INIT);
  cholqr2<L>(w, dwl, W.as<double>(), dptrs, V1, R0.as<double>(), -1);
  hipLaunchKernelGGL((k_ext_gamma<L>), dim3(1), dim3(64), 0, st, R0.as<double>(), S, gamma.as<double>());
  kt.collect();
  {
    int f[2];
    std::vector<double> g(LL);
    LYAP_HIP(hipMemcpyAsync(g.data(), gamma.p, LL * sizeof(double), hipMemcpyDeviceToHost, st));
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
    out->beta = std::sqrt(tr);  // ||C||_F = ||gamma||_F
  }
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
    ck.run(band.as<double>(), mm * L, gamma.as<double>(), taulog.as<double>() + (size_t)(mm - 1) * LL,
           chk.as<CheckOut>());
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
    const int j = m;  // current block V_j (0-based)
    const double* Vj = V[j].as<double>();
    launch_apply<double>(op.dev, L, Vj, AV.as<double>(), eg, st);
    hipLaunchKernelGGL((k_ext_split<S>), dim3(eg), dim3(kBlock), 0, st, Vj, n, Bs.as<double>());
    cg.solve(Bs.as<double>(), Xs.as<double>(), &kt);
    kt.mark(LYAP_K_EXT_ORTH);
    hipLaunchKernelGGL((k_ext_merge<S>), dim3(eg), dim3(kBlock), 0, st, AV.as<double>(), L, Xs.as<double>(), n,
                       W.as<double>());
    for (int sweep = 0; sweep < 2; ++sweep) {
      gram<L>(w, dptrs, j + 1, W.as<double>());
      hipLaunchKernelGGL((k_ext_update<L>), dim3(w.G), dim3(kExtThreads), 0, st, dptrs, j + 1, w.H.as<double>(),
                         W.as<double>(), n);
      LYAP_LAUNCHED("k_ext_update");
    }
    double* Vn = new_block();
    cholqr2<L>(w, dwl, W.as<double>(), dptrs + j + 1, Vn, w.small.as<double>() + 8 * LL, j + 1);
    gram<L>(w, dptrs + j, 2, AV.as<double>());
    hipLaunchKernelGGL((k_ext_tband<L>), dim3(1), dim3(64), 0, st, w.H.as<double>(), band.as<double>(), j,
                       taulog.as<double>());
    LYAP_LAUNCHED("k_ext_tband");
    ++m;
    if (m == next_check || m == maxit) {
      int f[2];
      read_flags(f);
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
  LYAP_HIP(hipMemcpyAsync(tau_h.data(), taulog.as<double>() + (size_t)(m - 1) * LL, LL * sizeof(double),
                          hipMemcpyDeviceToHost, st));
  LYAP_HIP(hipStreamSynchronize(st));
  double tau_f = 0.0;
  for (double v : tau_h) tau_f += v * v;
  tau_f = std::sqrt(tau_f);
  double eps = o.trunc_eps;
  if (!(eps >= 0.0)) eps = std::min(1e-12, 0.05 * o.tol / (lam_absmax + tau_f)) * beta2;
  out->trunc_eps = eps;
  DevBuf M;
  kt.mark(LYAP_K_FINAL);
  const int t = finalise_factor(ck, band.as<double>(), gamma.as<double>(), eps, M, st);
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
    for (int i = 0; i < m; ++i) bp.push_back(V[i].p);
    kt.mark(LYAP_K_ZFLUSH);
    launch_zflush<double>(bp.data(), m, n, L, M.as<double>(), t, out->Z, n, 0, st);
  }
  LYAP_HIP(hipStreamSynchronize(st));
  kt.collect();
  const double z_ms = ms_since(t_z);

  if (o.want_T) {
    const int k = m * L;
    out->T_band = (double*)std::malloc((size_t)(L + 1) * k * sizeof(double));
    LYAP_HIP(hipMemcpy(out->T_band, band.p, (size_t)(L + 1) * k * sizeof(double), hipMemcpyDeviceToHost));
    for (int c = 0; c < k; ++c)
      for (int d = 0; d <= L; ++d)
        if (c + d >= k) out->T_band[(size_t)c * (L + 1) + d] = 0.0;
    std::vector<double> g(LL);
    LYAP_HIP(hipMemcpy(g.data(), gamma.p, LL * sizeof(double), hipMemcpyDeviceToHost));
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
  for (int i = 0; i < 12; ++i) {
    out->kern_ms[i] = kt.ms[i];
    out->kern_n[i] = kt.n[i];
  }
  {
    const double coef = op.coef_bytes_per_row();
    // CG direction: r, M^{-1}, p_old in, p, q out (+ coefficients); update: x, r, p, q, M^{-1} in, x, r out
    out->kern_bytes[LYAP_K_CG_DIR] = (double)n * (5.0 * S * 8 + 8 + coef);
    out->kern_bytes[LYAP_K_CG_UPD] = (double)n * (6.0 * S * 8 + 8);
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

}  // namespace lyap
